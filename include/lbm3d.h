/*
 * lbm3d.h -- C ABI of the D3Q19 and D3Q27 lattices: the BGK collide-and-
 * stream sweep with the non-reflective NSBC boundary of Euser & Vuik
 * (arXiv 2005.08674, Secs. 3 and 5) carried to three dimensions.
 *
 * D3Q19: c_0 = 0 (w 1/3); the six axis directions +x, -x, +y, -y, +z, -z
 * (w 1/18); the twelve face diagonals (w 1/36) in opposite pairs (1,1,0),
 * (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1), (1,0,-1), (-1,0,1),
 * (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1).  D3Q27: the same 19 (weights
 * 8/27, 2/27, 1/54) followed by the eight cube diagonals (w 1/216) in
 * opposite pairs (1,1,1), (-1,-1,-1), (1,1,-1), (-1,-1,1), (1,-1,1),
 * (-1,1,-1), (-1,1,1), (1,-1,-1).  c_s^2 = 1/3.  Equilibrium eq. feq_1,
 * collision eq. lbe_1, pull streaming eq. lbe_0.
 *
 * NSBC in 3-D: a node on k NSBC faces (k = 1 face, 2 edge, 3 corner) takes
 * the normalised sum of the faces' outward normals as its normal, so eq.
 * nes_2 reads m_p = m_b - (gamma / sqrt k) sum_j (m_b - m_{b - n_j}) with
 * first-order one-sided differences at time t; eq. nes_3 blends the far
 * field, eqs. nes_0/nes_1 rebuild every population whose pull source lies
 * outside the lattice (f^eq_i(m_c) + f_opp - f^eq_opp(m_c), or f^eq_i(m_c)
 * when the opposite is unknown too), and eq. nes_4 shifts all q of them by
 * w_i (drho + c_i . dj / c_s^2) so the node carries m_c.
 *
 * Memory: all device memory belongs to the caller (a workspace of
 * lbm3d_workspace_bytes); the context is a host object.  Population i of
 * node (x, y, z) is stored as the deviation f_i - w_i rho0 (encoded in the
 * storage format) in q planes of [nz][ny][pitch].  Calls return 0 or a negative LBM_ERR_* code (lbm.h) and
 * never abort; lbm_last_error() describes the last failure.  Work is
 * asynchronous on the stream given at init.
 */
#ifndef LBM3D_H
#define LBM3D_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm3d_ctx lbm3d_ctx;

enum { LBM3D_D3Q19 = 0, LBM3D_D3Q27 = 1 };

typedef struct {
    int32_t nx, ny, nz;   /* each >= 3, nx * ny * nz <= 2^28, and a plane with rows padded to
                             256 bytes (ny * nz * that row) under 4 GiB */
    double tau;           /* BGK relaxation time, > 0.5 */
    double rho0;          /* base density of the deviation form, > 0 */
    int32_t bc[6];        /* LBM_BC_PERIODIC or LBM_BC_NSBC per face: x = 0, x = nx-1, y = 0,
                             y = ny-1, z = 0, z = nz-1; periodic faces come in pairs */
    double gamma;         /* eq. nes_2 */
    int32_t store;        /* LBM_STORE_F64, LBM_STORE_F32, LBM_STORE_F16DEV or LBM_STORE_BF16DEV
                             (FP32 arithmetic for the last three; the 16-bit formats store
                             g_i / w_i, FP16 also scaled by 2^k, k chosen at init so the largest
                             initial value is about 2^12, as in lbm.h) */
    int32_t velocity_set; /* LBM3D_D3Q19 (q = 19) or LBM3D_D3Q27 (q = 27) */
} lbm3d_params;

/* Defaults: 3x3x3, tau 0.6, rho0 1, NSBC on all faces, gamma 0.6, FP32, D3Q19. */
int lbm3d_params_default(lbm3d_params* p);

/* Device workspace in bytes: two population buffers of q planes, two small
 * buffers of moments of the nodes next to the x faces, and 1.25 KiB of
 * scratch (a flag, the FP16 exponent reduction). */
int lbm3d_workspace_bytes(const lbm3d_params* p, size_t* bytes);

/* Create a context on `workspace` (device memory of at least
 * lbm3d_workspace_bytes bytes, 256-byte aligned, borrowed until
 * lbm3d_destroy) and set every node to f^eq of the initial fields: device
 * float64 arrays [nz][ny][nx] of rho - rho0, ux, uy, uz.  The far field starts
 * at beta = 0, m0 = (rho0, 0, 0, 0). */
int lbm3d_init(lbm3d_ctx** out, const lbm3d_params* p, void* workspace, size_t bytes, const double* drho,
               const double* ux, const double* uy, const double* uz, void* hip_stream);

/* Far-field criterion, eq. nes_3: beta in [0, 1], m0 = (rho, ux, uy, uz). */
int lbm3d_set_farfield(lbm3d_ctx* ctx, double beta, double rho, double ux, double uy, double uz);

/* Advance n >= 0 steps, one kernel launch per step. */
int lbm3d_step(lbm3d_ctx* ctx, int32_t n);

/* Moments into device float64 out[4][nz][ny][nx]: rho - rho0, ux, uy, uz. */
int lbm3d_moments(lbm3d_ctx* ctx, double* out);

/* Steps taken. */
int lbm3d_time(const lbm3d_ctx* ctx, int64_t* t);

/* FP16 scale exponent k in use (0 for the other formats). */
int lbm3d_f16_exp(const lbm3d_ctx* ctx, int32_t* k);

/* Checkpoint and restore: the state (the post-collision populations of the
 * current time, f_i - w_i rho0) to or from a device float64 [q][nz][ny][nx]
 * array.  Setting also refreshes the x-face moments the next step reads.
 * Asynchronous. */
int lbm3d_get_populations(lbm3d_ctx* ctx, double* out);
int lbm3d_set_populations(lbm3d_ctx* ctx, const double* in);

/* *ok = 1 if every stored population is finite, else 0 (and the call returns
 * LBM_ERR_NONFINITE).  Synchronizes the stream. */
int lbm3d_check_finite(lbm3d_ctx* ctx, int* ok);

/* Launch shapes of the step kernel: a block of BX x BY threads owns a
 * BX x BY column of nodes and marches through ZC consecutive z-planes
 * ("BXxBYxzZC", "+ntl" when the pulls are loaded non-temporally); the
 * blocks' columns are cut into eight contiguous stretches, one per XCD, so
 * that x-neighbouring blocks, which share the cache lines their shifted
 * pulls straddle, run on one L2.  The "pair:BXxBYxzZC" shapes (ids after the
 * others) give each thread two x-neighbouring nodes and move both nodes'
 * value of a population with one 32-bit load or store; they take FP16 and
 * BF16 storage with non-periodic x faces and an even nx only (lbm3d_set_shape
 * fails otherwise).  All shapes give identical results.
 * lbm3d_shape_describe names candidate `id`; lbm3d_set_shape selects one
 * (default 128x1xz1); lbm3d_autotune times each shape the lattice takes
 * (median of `reps` launches after a warm-up; the state is not advanced),
 * keeps the fastest and writes its id to *best and, if times_ms is not NULL,
 * one median per shape (-1 for shapes the lattice does not take). */
int lbm3d_shape_count(void);
int lbm3d_shape_describe(int32_t id, char* buf, size_t len);
int lbm3d_set_shape(lbm3d_ctx* ctx, int32_t id);
int lbm3d_autotune(lbm3d_ctx* ctx, int32_t reps, int32_t* best, float* times_ms);

/* Release the context (waits for its stream). */
void lbm3d_destroy(lbm3d_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM3D_H */
