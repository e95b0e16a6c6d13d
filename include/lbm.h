/*
 * lbm.h -- C ABI of the MI355X (gfx950) D2Q9 lattice-Boltzmann library with
 * the Non-equilibrium Symmetry Boundary Condition (NSBC) of Euser & Vuik,
 * "A non-reflective boundary condition for LBM based on the assumption of
 * non-equilibrium symmetry" (arXiv 2005.08674).
 *
 * The problem the calls solve (paper Secs. 3 and 5): a D2Q9 lattice (Fig. 1)
 * evolves by the lattice Boltzmann equation (eq. lbe_0) with the BGK
 * collision (eqs. lbe_1, feq_1) and relaxation time tau; on the edges marked
 * NSBC the incoming populations are rebuilt from a predicted macroscopic vector
 * (eqs. nes_0..nes_4) with relaxation parameter gamma, far-field factor beta
 * and reference vector m0; the observable is (rho, u) (eqs. cf_0, cf_1).
 *
 * Conventions shared by every call
 *  - Lattice directions are numbered as in Fig. 1: c_0 = (0,0), c_1 = (1,0),
 *    c_2 = (-1,0), c_3 = (0,1), c_4 = (0,-1), c_5 = (1,1), c_6 = (-1,-1),
 *    c_7 = (-1,1), c_8 = (1,-1).  Node (x, y): x in [0, nx), y in [0, ny), y up.
 *  - Fields exchanged with the caller are row-major [ny][nx] arrays in DEVICE
 *    memory (x fastest).  Densities are exchanged as the deviation rho - rho0.
 *  - Stored populations are deviations g_i = f_i - f^eq_i(rho0, u_b) from the
 *    discrete equilibrium of a base state (rho0, u_b); u_b = 0 (the default)
 *    gives g_i = f_i - w_i rho0.  A base velocity equal to the mean flow keeps
 *    the stored values, and their rounding errors, proportional to the
 *    disturbance instead of to the mean flow.
 *  - All device memory is owned by the caller; the library never allocates
 *    device memory.  Contexts are host objects owned by the library.
 *  - Every call returns LBM_OK (0) or a negative LBM_ERR_* code and never
 *    aborts.  Argument errors are reported before anything is enqueued.
 *    lbm_last_error() returns a message for the calling thread's last error.
 *  - Work is enqueued asynchronously on the HIP stream given to lbm_init; a
 *    call that returns data to the host says so and synchronizes that stream.
 *  - One context may be used from one thread at a time.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBM_OK = 0,
    LBM_ERR_ARG = -1,         /* invalid argument or parameter combination */
    LBM_ERR_HIP = -2,         /* a HIP runtime call or kernel launch failed */
    LBM_ERR_STATE = -3,       /* call not valid in the context's current state */
    LBM_ERR_NONFINITE = -4,   /* the populations hold a NaN or infinity */
    LBM_ERR_UNSUPPORTED = -5  /* valid request the library does not implement */
};

/* Edge index in lbm_params.bc: 0 = left (x = 0), 1 = right (x = nx-1),
 * 2 = bottom (y = 0), 3 = top (y = ny-1).
 * LBM_BC_PERIODIC: wrap-around (edges come in pairs).
 * LBM_BC_NSBC: the non-reflective boundary of Sec. 5 (eqs. nes_0..nes_4).
 * LBM_BC_VELOCITY: a Dirichlet velocity edge, the inlet of the paper's test
 *   case 2 (Sec. 7, which only cites the scheme): the node takes the velocity
 *   set by lbm_set_velocity_edge and the density its known populations fix,
 *   rho_w = (sum_{c.n = 0} f + 2 sum_{c.n > 0} f) / (1 + u_w.n) with n the
 *   outward normal, then the incoming populations and the correction of eqs.
 *   nes_1 and nes_4 at (rho_w, u_w).  Left and right edges only, with
 *   periodic bottom and top (no corners). */
enum { LBM_BC_PERIODIC = 0, LBM_BC_NSBC = 1, LBM_BC_VELOCITY = 2 };

/* Storage of the populations.  Arithmetic is fp64 for LBM_STORE_F64 and fp32
 * for the three others.  The 16-bit codecs store s_i = g_i / w_i * 2^k with
 * round-to-nearest-even: k = lbm_params.f16_exp for FP16 (a per-lattice power
 * of two that keeps s_i in FP16's normal range), k = 0 for BF16. */
enum { LBM_STORE_F64 = 0, LBM_STORE_F32 = 1, LBM_STORE_F16DEV = 2, LBM_STORE_BF16DEV = 3 };

/* Collision model (lbm_params.collision).
 * LBM_COLL_BGK: single relaxation time, eq. lbe_1 (Sec. 3), rate 1/tau.
 * LBM_COLL_MRT: multiple relaxation times, eqs. mrt_lbe, mrt_vm, mrt_rm
 *   (Sec. 4): f* = f - M^-1 S (M f - M f^eq), the rows of M the Gram-Schmidt
 *   orthogonalisation of the moments 1, |c|^2, |c|^4, c_x, c_x|c|^2, c_y,
 *   c_y|c|^2, c_x^2 - c_y^2, c_x c_y, and
 *   S = diag(0, omega_e, omega_eps, 0, omega_q, 0, omega_q, 1/tau, 1/tau):
 *   the viscous rate is 1/tau and density and momentum are not relaxed. */
enum { LBM_COLL_BGK = 0, LBM_COLL_MRT = 1 };

/* lbm_params.f16_exp value asking lbm_init to choose k from the initial
 * fields so that max |g_i / w_i| * 2^k is close to 2^12. */
#define LBM_F16_EXP_AUTO (-1000)

typedef struct lbm_ctx lbm_ctx;

typedef struct {
    int32_t nx, ny;       /* lattice size, each >= 3 */
    double tau;           /* relaxation time, dt = 1: BGK's (eq. lbe_1), > 0.5; or MRT's viscous
                             rate omega_nu = 1/tau (eq. mrt_rm), >= 0.5 (0.5: zero viscosity) */
    double rho0;          /* base density of the deviation form, > 0 */
    int32_t bc[4];        /* LBM_BC_* per edge; periodic edges come in pairs (left+right, bottom+top) */
    double gamma;         /* NSBC relaxation parameter, eq. nes_2 (the paper uses 0.6) */
    int32_t store;        /* LBM_STORE_* */
    int32_t corr_mode;    /* eq. nes_4: 0 = shift w_i (drho + c_i.dj / c_s^2) (exact moments),
                             1 = literal w_i (drho + c_i.dj) */
    int32_t grad_order;   /* eq. nes_2 normal derivative: 1 = two-point, 2 = three-point one-sided */
    int32_t corner_mode;  /* corner nodes of two NSBC edges: 0 = diagonal normal (gamma/sqrt 2),
                             1 = gamma/2 */
    int32_t f16_exp;      /* k of the FP16 codec, or LBM_F16_EXP_AUTO; ignored by other stores */
    int32_t collision;    /* LBM_COLL_BGK (default) or LBM_COLL_MRT */
    double ubase[2];      /* base velocity u_b of the deviation form, |u_b| <= 0.5 (default 0) */
    double omega_e;       /* MRT rates of the energy, energy-square and energy-flux moments */
    double omega_eps;     /* (eq. mrt_rm), each in (0, 2]; ignored by BGK; default 1.9 */
    double omega_q;
} lbm_params;

/* Fill *p with defaults: 3x3 lattice, tau 0.6, rho0 1, NSBC on all edges,
 * gamma 0.6, FP32 storage, corr_mode 0, grad_order 1, corner_mode 0,
 * f16_exp auto, u_b = 0, BGK collision (MRT rates 1.9 when MRT is chosen).
 * Always succeeds for a non-null p. */
int lbm_params_default(lbm_params* p);

/* Device workspace, in bytes, that lbm_init needs for these parameters: two
 * population buffers (9 planes each) and a scratch area for reductions. */
int lbm_workspace_bytes(const lbm_params* p, size_t* bytes);

/* Create a context on `workspace` (device memory of at least
 * lbm_workspace_bytes bytes, 256-byte aligned, borrowed until lbm_destroy)
 * and set every node to the discrete equilibrium of the initial fields
 * (f = f^eq(rho, u), eq. feq_1).  drho, ux, uy are device float64 [ny][nx]
 * arrays (rho - rho0 and the velocity).  `hip_stream` is the hipStream_t all
 * later work of this context is enqueued on (NULL = the null stream).
 * Synchronizes the stream (it reads a reduction back when f16_exp is auto).
 * The far-field factor starts at beta = 0 with m0 = (rho0, 0, 0).
 * The 16-bit stores hold s_i = g_i / w_i * 2^k (see LBM_STORE_*). */
int lbm_init(lbm_ctx** out, const lbm_params* p, void* workspace, size_t bytes,
             const double* drho, const double* ux, const double* uy, void* hip_stream);

/* Far-field criterion, eq. nes_3: m_c = (1 - beta) m_p + beta m0 with
 * m0 = (rho_ref, ux_ref, uy_ref) (absolute density).  beta in [0, 1].
 * Takes effect from the next step. */
int lbm_set_farfield(lbm_ctx* ctx, double beta, double rho_ref, double ux_ref, double uy_ref);

/* Velocity u_w = (ux, uy) of the lattice's LBM_BC_VELOCITY edges (both take
 * the same one), |u_w| <= 0.5; (0, 0) after lbm_init.  Takes effect from the
 * next step. */
int lbm_set_velocity_edge(lbm_ctx* ctx, double ux, double uy);

/* Advance n >= 0 time steps (stream, NSBC, collide; eqs. lbe_0, nes_0..nes_4,
 * lbe_1).  Asynchronous; the context's time advances by n.  The call is a
 * roctx range named "lbm_step" (as are the other stepping and tuning calls,
 * each under its own name), visible to rocprofv3 --marker-trace. */
int lbm_step(lbm_ctx* ctx, int32_t n);

/* Moments of every node at the current time (eqs. cf_0, cf_1): writes
 * rho - rho0 (deviation = 1) or rho (deviation = 0) to drho_out and the
 * velocity to ux_out, uy_out, each a device [ny][nx] array of float64
 * (out_f64 = 1) or float32 (out_f64 = 0).  Any output pointer may be NULL
 * to skip it.  Asynchronous. */
int lbm_moments(lbm_ctx* ctx, void* drho_out, void* ux_out, void* uy_out, int out_f64, int deviation);

/* Current time step count. */
int lbm_time(const lbm_ctx* ctx, int64_t* t);

/* Message of the calling thread's last failed call ("" if none).  The
 * pointer stays valid until the next library call on the same thread. */
const char* lbm_last_error(void);

/* Release the context.  The workspace is the caller's and is not freed.
 * Waits for the context's stream. */
void lbm_destroy(lbm_ctx* ctx);

/* ---------------------------------------------------------------- extras */

/* Decoded populations as f_i - w_i rho0 (whatever the base velocity) in a
 * device float64 [9][ny][nx] array.  Asynchronous. */
int lbm_get_populations(lbm_ctx* ctx, double* g_out);

/* Overwrite the state with the device float64 [9][ny][nx] values
 * g_i = f_i - w_i rho0 (converted to the base state and encoded to the
 * context's storage).  The state is the post-collision
 * population set, the quantity lbm_get_populations returns.  Asynchronous. */
int lbm_set_populations(lbm_ctx* ctx, const double* g);

/* *ok = 1 if every stored population is finite, else 0 (and the call returns
 * LBM_ERR_NONFINITE).  Synchronizes the stream. */
int lbm_check_finite(lbm_ctx* ctx, int* ok);

/* Checkpoint of the whole state as host bytes, for continuing a run in a
 * later process (the paper's state at time t is the population set, Sec. 3,
 * eq. lbe_0, plus the far-field criterion of eq. nes_3).
 * lbm_save_bytes: the size lbm_save writes, 256 + 9 * nx * ny * (bytes per
 * stored population).
 * lbm_save: writes into host_buf (>= that size, caller-owned) a 256-byte
 * header -- magic "LBMCKPT1", version 1, lattice size, storage and FP16
 * exponent, edges, NSBC readings, collision model and rates, tau, rho0, u_b,
 * gamma, the time step t, the far-field factor beta and vector m0, the
 * velocity-edge velocity u_w, the closure mode with the byte count and
 * 64-bit FNV-1a hash of the network the context uses, and the payload's
 * size and hash -- followed by the populations exactly as stored, as a
 * compact [9][ny][nx] array in the storage format.  Synchronizes the stream.
 * lbm_load: restores such a checkpoint into a context created with the same
 * lattice size, storage, edges, readings, collision model and rates, tau,
 * rho0, u_b and gamma (else LBM_ERR_STATE) and using the same closure
 * network, or none, as the saved one (else LBM_ERR_STATE); a damaged or
 * foreign buffer gives LBM_ERR_ARG.  It sets the populations, t, beta, m0,
 * u_w and, for FP16 storage, the codec exponent the values were saved with,
 * so the run continues bit for bit as the saved one would have.  A refused
 * checkpoint leaves the context unchanged.  Synchronizes the stream. */
int lbm_save_bytes(const lbm_ctx* ctx, size_t* bytes);
int lbm_save(lbm_ctx* ctx, void* host_buf, size_t bytes);
int lbm_load(lbm_ctx* ctx, const void* host_buf, size_t bytes);

/* Debug mode.  level 0: off.  level 1: every call of this library that
 * enqueues work on a stream synchronizes that stream before returning and
 * reports a failed kernel or HIP call as LBM_ERR_HIP with the call's name in
 * lbm_last_error().  level 2: in addition every step call checks that the
 * populations are finite and returns LBM_ERR_NONFINITE when they are not.
 * The initial level is read once from the environment variable LBM_DEBUG
 * ("0", "1" or "2"; unset = 0); lbm_set_debug changes it for the whole
 * process (level in [0, 2], else LBM_ERR_ARG). */
int lbm_set_debug(int32_t level);
int lbm_debug_level(int32_t* level);

/* FP16 codec exponent k in use (0 for the other stores). */
int lbm_f16_exp(const lbm_ctx* ctx, int32_t* k);

/* Acoustic energy of a perturbation, in fp64 with a fixed-order reduction:
 *   E = sum over the nodes of `test` of 1/2 [c_s^2 d_rho^2 / rho0 + rho0 |d_u|^2]
 * where (d_rho, d_u) is the difference between `test` at node (x, y) and
 *  - `ref` at node (x + x_off, y + y_off) when ref is not NULL (a larger
 *    reference lattice containing test's window; both must share rho0 and
 *    the window must fit inside ref), or
 *  - the uniform state (rho0, ux_ref, uy_ref) when ref is NULL.
 * The result is written to *out_dev, one float64 in device memory.
 * Asynchronous on test's stream; when ref is given its stream must be the same
 * stream or the caller orders the two. */
int lbm_energy(lbm_ctx* test, const lbm_ctx* ref, int32_t x_off, int32_t y_off,
               double ux_ref, double uy_ref, double* out_dev);

/* lbm_energy without the context's workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same value, bit for bit,
 * computed by the same kernels, whose 1024 fp64 block partials go to a
 * static 8 KiB device array of the library instead of the workspace.  The
 * call allocates nothing.  Each GPU holds one such array for the life of
 * the process, looked up at lbm_init (or the first call on a device); every
 * call on a GPU reuses it and each call overwrites all of it, so calls that
 * overlap on one GPU (different streams, no ordering) race and must be
 * serialized by the caller.  The contexts' device must be current
 * (LBM_ERR_ARG otherwise); a reduction needing more partials than the array
 * holds is refused with LBM_ERR_UNSUPPORTED.  Asynchronous on test's
 * stream, as lbm_energy. */
int lbm_energy_noalloc(lbm_ctx* test, const lbm_ctx* ref, int32_t x_off, int32_t y_off,
                       double ux_ref, double uy_ref, double* out_dev);

/* Bulk-kernel tile shapes.  lbm_tile_count gives the number of candidate
 * shapes; lbm_tile_describe writes a short text name of candidate `id` into
 * buf; lbm_set_tile selects one for this context (the default is chosen from
 * the lattice and storage).  lbm_autotune times every candidate on the
 * context's own lattice as lbm_step launches it (the fused step launch, or,
 * with the closure or fusion off, the bulk kernel followed by the edge
 * kernel: whole steps either way), `reps` timed runs of 24 consecutive
 * steps each, median of those, after one warm-up, and selects the fastest.
 * The launches are consecutive steps, as stepping runs them (a launch repeated on one
 * unchanged buffer can be served from the GPU's last-level cache, 256 MB on
 * MI355X, where two buffers would not fit): the state is saved to a
 * temporary device copy (one buffer's size, allocated and freed here) and
 * restored afterwards, so it and t are left unchanged.  It writes the chosen
 * id to *best and, if times_ms is not NULL,
 * the per-candidate median step time in milliseconds (length
 * lbm_tile_count).  Synchronizes the stream. */
int lbm_tile_count(void);
int lbm_tile_describe(int32_t id, char* buf, size_t len);
int lbm_set_tile(lbm_ctx* ctx, int32_t id);
int lbm_get_tile(const lbm_ctx* ctx, int32_t* id);
int lbm_autotune(lbm_ctx* ctx, int32_t reps, int32_t* best, float* times_ms);

/* Per-kernel timing with HIP events on the context's stream.  While enabled,
 * every lbm_step launch of the bulk kernel and of the edge kernel is
 * bracketed by events; lbm_kernel_times synchronizes the stream and returns
 * the summed elapsed milliseconds and launch counts since the last reset.
 * With the fused step launch (lbm_set_fused) each step is one launch, counted
 * as a bulk launch; the edge count then stays 0. */
int lbm_enable_timing(lbm_ctx* ctx, int on);
int lbm_kernel_times(lbm_ctx* ctx, double* bulk_ms, int64_t* bulk_launches,
                     double* edge_ms, int64_t* edge_launches);

/* Run the edge/corner kernel on a second stream of the library's own,
 * concurrently with the bulk kernel of the same step (on = 1), or after it on
 * the context's stream (on = 0, the default: on gfx950 the extra event
 * traffic of the overlapped form costs more than the edge kernel it hides).  Both orders give identical
 * results: within a step the two kernels read the same buffer and write
 * disjoint nodes; every step waits for both kernels of the previous one, and
 * lbm_step returns with the context's stream ordered after all its work. */
int lbm_set_overlap(lbm_ctx* ctx, int on);

/* Bytes the bulk kernel must move per node and step (2 x 9 x bytes per
 * stored population) and the node count it updates per launch: the interior
 * (nx-2)(ny-2), or all nx*ny nodes with the fused step launch. */
int lbm_bulk_traffic(const lbm_ctx* ctx, int64_t* bytes_per_node, int64_t* nodes_per_launch);

/* on = 1 (the default): each single step is ONE launch whose first blocks
 * run the edge/corner segments and the rest the bulk tiles, so the edge work
 * overlaps the bulk stream instead of following it; results are identical to
 * the two separate launches.  on = 0: separate edge and bulk launches.  The
 * closure and the overlap option always use separate launches. */
int lbm_set_fused(lbm_ctx* ctx, int on);

/* Multi-step sweeps: for lattices with NSBC on all four edges, one launch
 * advances two (t -> t + 2) or three (t -> t + 3) time steps.  Two-step
 * shapes: each block computes level t + 1 on its 64 x TY tile plus a
 * margin, keeps it in LDS, and computes level t + 2 on the tile from there.
 * Three-step shapes keep levels t + 1 and t + 2 in LDS (margins 2 and 1
 * around whole 64 x TY tiles: the last tile of a row or column overlaps its
 * neighbour), and need nx >= 64, ny >= TY and, for FP64, TY <= 12.  Either
 * way the state crosses HBM about once per launch (2 x 9 x bytes per stored
 * population per node, plus margins re-read from L2), and results are
 * bit-identical to single steps: intermediate levels are held in the
 * storage format exactly as a store would write them.  Column-march shapes
 * ("...+march<MR>xh<H>..."): one launch runs the edge tiles (the ring of
 * 64 x TY tiles around the inner tiles' rectangle) as tiles and the inner
 * rectangle as 64-column strips cut into chunks of about H rows, each
 * walked down in rounds of MR rows with every intermediate level's last
 * MR + 2 rows in an LDS ring, so no row margin is recomputed; same
 * conditions and results as the tile shapes of that TY.  They are single-
 * lattice shapes (lbm_ens_set_two_step refuses them).
 * lbm_two_step_count / lbm_two_step_describe ("2step:..." or "3step:...")
 * list the candidate shapes and lbm_two_step_steps gives a shape's steps per
 * launch; lbm_set_two_step selects one (-1 turns the sweeps off, the
 * default) and fails for lattices it does not support.  With a shape
 * selected, lbm_step advances groups of that many steps with it; after
 * three-step launches a remainder of two steps takes one two-step launch
 * (the best two-step shape lbm_autotune_two_step timed, else a default per
 * storage format), any other remainder single-step launches.  With the
 * learned closure on (lbm_set_closure) the three-step shapes carry it: in
 * their edge tiles the network corrects m_c of every single-normal edge
 * node at each of the three levels, from the previous level, as the
 * single-step edge kernel does (bit-identical to closure single steps; the
 * edge tiles then run in a kernel of their own on a second stream beside
 * the inner tiles or strips; each launch's edge-tile kernel waits only for
 * the previous launch's inner part, and before lbm_step returns the stream
 * has waited for the last of them); two-step shapes and remainders then run
 * as closure single steps.  The
 * overlap option and periodic edges always use the single-step kernels.
 * lbm_autotune_two_step times every shape the lattice supports (`reps`
 * runs of consecutive launches covering at least 24 steps each, median,
 * from a saved and restored state as lbm_autotune does; the state is left
 * unchanged), selects the one with
 * the least time per step, writes its id to *best and, if times_ms is not
 * NULL, per shape the median run time divided by its steps
 * (ms per step; -1 for shapes the lattice cannot take).  Synchronizes the
 * stream.  lbm_two_step_times returns the summed elapsed milliseconds and
 * the count of multi-step launches timed while lbm_enable_timing is on, and
 * resets them. */
int lbm_two_step_count(void);
int lbm_two_step_describe(int32_t id, char* buf, size_t len);
int lbm_two_step_steps(int32_t id, int32_t* steps);
int lbm_set_two_step(lbm_ctx* ctx, int32_t id);
int lbm_get_two_step(const lbm_ctx* ctx, int32_t* id);
int lbm_autotune_two_step(lbm_ctx* ctx, int32_t reps, int32_t* best, float* times_ms);
int lbm_two_step_times(lbm_ctx* ctx, double* ms, int64_t* launches);

/* Plain device-to-device copy of `bytes` bytes (16-byte loads, non-temporal
 * stores) on `hip_stream`: the streaming-bandwidth reference the bulk kernel
 * is measured against, and the known-size kernel used to calibrate hardware
 * byte counters.  src and dst are 16-byte aligned, non-overlapping device
 * buffers owned by the caller.  Asynchronous. */
int lbm_stream_copy(const void* src, void* dst, size_t bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
