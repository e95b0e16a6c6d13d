/*
 * lbm_ensemble.h -- C ABI of the batched ensemble: many independent D2Q9
 * BGK + NSBC lattices of different sizes and parameters advanced together.
 *
 * The method per lattice is the one of lbm.h (Euser & Vuik, arXiv 2005.08674,
 * Secs. 3 and 5: eqs. lbe_0, lbe_1, feq_1, nes_0..nes_4).  The ensemble adds
 * no arithmetic: one launch of the bulk kernel covers the interior tiles of
 * every member (through a device table of {member, tile}), one launch of the
 * edge kernel covers the edge segments of every member, and n such steps can
 * be captured once into a HIP graph and replayed as a single graph launch.
 * Every member's result is bit-identical to the same lattice run alone
 * through lbm.h.
 *
 * Conventions are those of lbm.h: device memory belongs to the caller, the
 * ensemble object is host memory owned by the library, calls return LBM_OK or
 * a negative LBM_ERR_* code (message in lbm_last_error()), and work is
 * asynchronous on the caller's stream.
 */
#ifndef LBM_ENSEMBLE_H
#define LBM_ENSEMBLE_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ens lbm_ens;

/* Device workspace in bytes for `count` members described by members[0..count-1]
 * (each a valid lbm_params; all must use the same `store`): descriptor and
 * tile tables, a scratch area, and two population buffers per member. */
int lbm_ens_workspace_bytes(const lbm_params* members, int32_t count, size_t* bytes);

/* Create the ensemble on `workspace` (device memory, 256-byte aligned, at
 * least lbm_ens_workspace_bytes, borrowed until lbm_ens_destroy) and set
 * every member to the equilibrium of its initial fields (eq. feq_1).
 * drho, ux, uy are device float64 arrays holding the members' [ny][nx]
 * fields one after another (member m starts at element sum_{k<m} nx_k ny_k).
 * All members start with beta = 0, m0 = (rho0, 0, 0).  Synchronizes
 * `hip_stream` (the stream all later work goes to). */
int lbm_ens_init(lbm_ens** out, const lbm_params* members, int32_t count, void* workspace, size_t bytes,
                 const double* drho, const double* ux, const double* uy, void* hip_stream);

/* Far-field criterion of one member (eq. nes_3), as lbm_set_farfield.  Takes
 * effect from the next step, including steps of already captured graphs. */
int lbm_ens_set_farfield(lbm_ens* e, int32_t member, double beta, double rho_ref, double ux_ref, double uy_ref);

/* Velocity of one member's LBM_BC_VELOCITY edges, as lbm_set_velocity_edge.
 * Takes effect from the next step, including steps of captured graphs. */
int lbm_ens_set_velocity_edge(lbm_ens* e, int32_t member, double ux, double uy);

/* Advance every member n >= 0 steps: one launch per step (fused edge and
 * bulk work), two per step when fusion is off or a member runs the closure,
 * or one launch per 2 or 3 steps when a multi-step shape is set (the steps
 * left over at the end run singly). */
int lbm_ens_step(lbm_ens* e, int32_t n);

/* Floats per logged site: the closure inputs (LBM_MLP_INPUTS = 96), m_c - m0
 * and the strip amplitude A (4), and the residual target (3). */
#define LBM_ENS_LOG_FLOATS 103

/* Sites that lbm_ens_step_graph logs as closure training data (Sec. 5: the
 * boundary-strip moments that eq. nes_2 extrapolates, and the moments the
 * boundary node should carry one step later).  member_sites and twin_sites
 * are device int32 arrays [n][4] of rows (member, x, y, edge) as for
 * lbm_ens_closure_features: row i names a boundary node of a member and the
 * same physical node in a larger "twin" member run alongside it (the
 * reference whose moments are the target).  Borrowed until replaced; n = 0
 * clears them.  n <= 2^24. */
int lbm_ens_set_log_sites(lbm_ens* e, const int32_t* member_sites, const int32_t* twin_sites, int32_t n);

/* Bytes lbm_ens_step_graph writes when logging every log_every steps over n
 * steps: ceil(n / log_every) records of n_sites * LBM_ENS_LOG_FLOATS floats. */
int lbm_ens_log_bytes(const lbm_ens* e, int32_t n, int32_t log_every, size_t* bytes);

/* Advance every member n >= 1 steps with one launch of a HIP graph holding
 * the n steps' kernel launches.  The graph is captured and instantiated on
 * first use for these arguments (and step parity) and cached until
 * lbm_ens_destroy or a change of shape, fusion, multi-step shape or closure
 * set.
 * log_buf = NULL: the launches lbm_ens_step would issue.
 * log_buf != NULL (device, 16-byte aligned, >= lbm_ens_log_bytes bytes;
 * log sites set): at every step s = j * log_every (j = 0, 1, ...) of the run
 * the graph writes record j -- the closure inputs of the member sites at
 * time s ([n_sites][96] floats, as lbm_ens_closure_features), then their
 * m_c - m0 and A ([n_sites][4]), runs step s as one single step, and writes
 * the residual target at time s + 1 from the twin sites ([n_sites][3], as
 * lbm_ens_closure_moments with sub = that m_c) -- and advances the other
 * steps as lbm_ens_step would.  The records are exactly what those calls
 * return when issued between steps, so one graph launch generates a whole
 * round of training data. */
int lbm_ens_step_graph(lbm_ens* e, int32_t n, void* log_buf, size_t log_bytes, int32_t log_every);

/* on = 1 (the default): each step is one launch whose first blocks run the
 * members' edge segments and the rest their bulk tiles; on = 0: separate
 * bulk and edge launches.  Identical results either way.  Steps in which a
 * member runs the learned closure always use separate launches. */
int lbm_ens_set_fused(lbm_ens* e, int on);

/* Moments of one member, as lbm_moments. */
int lbm_ens_moments(lbm_ens* e, int32_t member, void* drho_out, void* ux_out, void* uy_out, int out_f64,
                    int deviation);

/* Populations of one member as f_i - w_i rho0, device float64 [9][ny][nx]. */
int lbm_ens_get_populations(lbm_ens* e, int32_t member, double* g_out);

/* Steps taken so far (the same for every member). */
int lbm_ens_time(const lbm_ens* e, int64_t* t);

/* Total node count, and the block counts of one bulk launch and of one edge
 * launch for the current tile shape. */
int lbm_ens_info(const lbm_ens* e, int64_t* nodes, int32_t* bulk_blocks, int32_t* edge_blocks);

/* Bulk tile shapes of the ensemble kernel, "BXxBYxNYT" (block BX x BY, NYT
 * nodes per thread along y).  lbm_ens_set_shape rebuilds the tile table and
 * work list (cached graphs are dropped).
 * lbm_ens_autotune times every shape as the launch a step uses (the fused
 * step, or the bulk kernel when fusion is off or a member runs the closure;
 * median of `reps` launches after one warm-up; the state is not advanced) and
 * keeps the fastest; times_ms (optional) receives one median per shape. */
int lbm_ens_shape_count(void);
int lbm_ens_shape_describe(int32_t id, char* buf, size_t len);
int lbm_ens_set_shape(lbm_ens* e, int32_t id);
int lbm_ens_autotune(lbm_ens* e, int32_t reps, int32_t* best, float* times_ms);

/* Multi-step sweeps over the whole ensemble (the single-lattice sweeps of
 * lbm_set_two_step, lbm.h: the intermediate levels of each 64 x TY tile kept
 * in LDS, eqs. lbe_0, lbe_1 / mrt_lbe and nes_0..nes_4 applied per level; results
 * bit-identical to single steps).  Shapes are the lbm_two_step_count /
 * lbm_two_step_describe candidates, two or three steps per launch
 * (lbm_two_step_steps); the ensemble lays every member's tiles out in one
 * list whose contiguous eighths run on the 8 XCDs (the shape's own block map
 * is not used).  lbm_ens_set_two_step selects a shape (-1, the default,
 * turns the sweeps off); LBM_ERR_UNSUPPORTED for the column-march shapes
 * (single lattices only) and unless every member has NSBC on all four edges
 * and, for a three-step shape, is at least 64 x its tile rows (FP64: tile
 * rows <= 12).  While a member runs the learned closure the
 * ensemble steps singly.  lbm_ens_autotune_two_step times every shape the
 * members take (median of `reps` launches, after one warm-up; the state is
 * not advanced), selects the one with the least time per step and writes its
 * id to *best and, if times_ms is not NULL, per shape the median launch time
 * divided by its steps per launch (ms per step; -1 for shapes the members
 * cannot take; length lbm_two_step_count).  Both drop cached graphs; the
 * autotuner synchronizes the stream. */
int lbm_ens_set_two_step(lbm_ens* e, int32_t id);
int lbm_ens_get_two_step(const lbm_ens* e, int32_t* id);
int lbm_ens_autotune_two_step(lbm_ens* e, int32_t reps, int32_t* best, float* times_ms);

/* Release the ensemble (waits for its stream; destroys cached graphs). */
void lbm_ens_destroy(lbm_ens* e);

#ifdef __cplusplus
}
#endif

#endif /* LBM_ENSEMBLE_H */
