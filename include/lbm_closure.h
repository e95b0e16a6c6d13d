/*
 * lbm_closure.h -- C ABI of the learned boundary closure: a small network
 * that replaces NSBC's prediction of the boundary macroscopic vector
 * (extrapolation, eq. nes_2, and far-field blend, eq. nes_3 -- Euser & Vuik,
 * arXiv 2005.08674, Sec. 5) by m_c + network correction, while NSBC itself
 * (assignment and correction, eqs. nes_0, nes_1, nes_4) stays as is and is
 * also the fallback.
 *
 * Network: 96 inputs (87 used) -> 64 tanh -> 64 tanh -> 3 outputs, BF16
 * weights and layer inputs, FP32 accumulation on gfx950 matrix cores.
 * Inputs of a boundary node b with outward normal n and tangent
 * t = (-n_y, n_x): for the nine strip nodes b - d n + k t (d = 0..2,
 * k = -1..1, node j = 3 d + k + 1 -> inputs 9 j .. 9 j + 8) the values
 * [rho - rho_ref, (u - u_ref).n, (u - u_ref).t, P_nn, P_nt, P_tt, Q_nnt,
 * Q_ntt, R_nntt], where (rho_ref, u_ref) is the far-field state m0 of
 * lbm_set_farfield and P, Q, R are the 2nd to 4th moments of f - f^eq in the
 * (n, t) frame; inputs 82..84 = NSBC's m_c - m0 as (drho, u.n, u.t).  These
 * 84 values are divided by the strip amplitude
 *   A = sqrt(mean over the 9 strip nodes of c_s^2 (rho - rho_ref)^2 / rho0^2
 *            + |u - u_ref|^2);
 * input 81 = 1/tau; inputs 85, 86 = u_ref.n, u_ref.t; inputs 87..95 = 0.
 * Inputs are then normalised by per-input mean and 1/std.  The 3 outputs,
 * times per-output scales and A, are added to m_c in the (n, t) frame, so
 * the correction scales with the disturbance and vanishes with it (A = 0
 * keeps m_c).
 *
 * All pointers are device memory owned by the caller unless marked host.
 * Return codes and asynchrony as in lbm.h.
 */
#ifndef LBM_CLOSURE_H
#define LBM_CLOSURE_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"
#include "lbm_ensemble.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_MLP_INPUTS 96
#define LBM_MLP_FEATURES 87
#define LBM_MLP_HIDDEN 64
#define LBM_MLP_OUTPUTS 3
/* packed fp32 parameters: W1 [64][96], b1 [64], W2 [64][64], b2 [64], W3 [3][64], b3 [3] */
#define LBM_MLP_NPARAM 10563

/* Size in bytes of the device network blob that lbm_mlp_export writes and
 * lbm_set_closure reads. */
int lbm_closure_net_bytes(size_t* bytes);

/* mode 1: every edge node with a single NSBC normal in the blob's regime
 * (kmin, see lbm_mlp_export) takes m_c + A times the network's correction (`net`, a blob from lbm_mlp_export, borrowed while in use);
 * corners, non-finite outputs and outputs beyond the blob's trust bound keep
 * NSBC's m_c.  mode 0: plain NSBC (net may be NULL). */
int lbm_set_closure(lbm_ctx* ctx, const void* net, int mode);

/* Training samples of one lattice at its current time.  sites: int32 [n][4]
 * rows (x, y, edge, 0) with edge 0..3 = outward normal (-1,0), (1,0), (0,-1),
 * (0,1); the strip b - d n + k t (d = 0..2, k = -1..1) must lie inside the
 * lattice.  feat_out: float [n][96] inputs before normalisation (already
 * divided by A); mc_out: float [n][4] = m_c - m0 as (rho, u.n, u.t), m_c
 * being NSBC's prediction with the lattice's gamma, beta, m0 and grad_order,
 * then A.  A site whose
 * strip leaves the lattice yields NaN rows.  Asynchronous. */
int lbm_closure_features(lbm_ctx* ctx, const int32_t* sites, int32_t n, float* feat_out, float* mc_out);

/* (rho - rho0, u.n, u.t) at the sites' nodes: m_out float [n][3].  With
 * `sub` (float [n][4], the mc_out of the previous step) the result is the
 * training residual (moments - m_c) / A instead, formed as
 * ((moments - m0) - (m_c - m0)) / A so that no large values cancel in fp32. */
int lbm_closure_moments(lbm_ctx* ctx, const int32_t* sites, int32_t n, const float* sub, float* m_out);

/* lbm_set_closure for one member of an ensemble, or for all of them when
 * member = -1. */
int lbm_ens_set_closure(lbm_ens* e, int32_t member, const void* net, int mode);

/* Ensemble versions: sites rows (member, x, y, edge); a row whose member is
 * not in [0, count) yields NaN. */
int lbm_ens_closure_features(lbm_ens* e, const int32_t* sites, int32_t n, float* feat_out, float* mc_out);
int lbm_ens_closure_moments(lbm_ens* e, const int32_t* sites, int32_t n, const float* sub, float* m_out);

/* ------------------------------------------------------------------ trainer */

typedef struct lbm_mlp lbm_mlp;

/* Workspace for batches of up to max_batch rows (a multiple of 64, <= 65536). */
int lbm_mlp_workspace_bytes(int32_t max_batch, size_t* bytes);

/* Trainer on `workspace`; params: packed fp32 initial parameters
 * (LBM_MLP_NPARAM).  Normalisation starts as the identity.  Synchronizes the
 * stream. */
int lbm_mlp_init(lbm_mlp** out, int32_t max_batch, void* workspace, size_t bytes, const float* params,
                 void* hip_stream);

/* Input mean / std and output scale (root mean square) from n training
 * samples: feat float [n][96] inputs, resid float [n][3] targets (true
 * next-step moments minus m_c, divided by A).  fp64 reduction in a fixed order.  Inputs
 * 87..95, constant inputs (spread below 1e-7 of the mean), and strip-node inputs whose standard deviation is
 * below 1e-3 of the largest standard deviation of the same moment over the
 * nine strip nodes (rounding noise of a moment that vanishes exactly, such as
 * the odd moments at the boundary row) get mean 0 and 1/std 0. */
int lbm_mlp_fit_normalization(lbm_mlp* m, const float* feat, const float* resid, int64_t n);

/* Normalise n samples: x_out BF16 [n][96] (round to nearest even), t_out
 * float [n][3] = resid / scale.  feat/resid as above; resid/t_out may be NULL. */
int lbm_mlp_pack(lbm_mlp* m, const float* feat, const float* resid, int64_t n, uint16_t* x_out, float* t_out);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, FP32 master weights) on
 * the mean squared error of `batch` samples; rows (int32 [batch], may be NULL
 * for 0..batch-1) selects them from x (BF16 [nsamples][96]) and t (float
 * [nsamples][3]); a row index outside [0, nsamples) counts as an empty
 * sample.  loss_out (device float, may be NULL) receives the batch loss
 * before the step.  Deterministic. */
int lbm_mlp_train_step(lbm_mlp* m, const uint16_t* x, const float* t, int64_t nsamples, const int32_t* rows,
                       int32_t batch, float lr, float* loss_out);

/* Gradients of the batch loss (packed like the parameters) without updating. */
int lbm_mlp_grads(lbm_mlp* m, const uint16_t* x, const float* t, int64_t nsamples, const int32_t* rows,
                  int32_t batch, float* grads_out, float* loss_out);

/* Network outputs y_out float [n][3] (normalised units) for n inputs. */
int lbm_mlp_forward(lbm_mlp* m, const uint16_t* x, int64_t n, float* y_out);

/* Current fp32 master parameters (packed). */
int lbm_mlp_params(lbm_mlp* m, float* params_out);

/* Normalisation in use: mean_out, inv_std_out float [96], scale_out float [3]. */
int lbm_mlp_normalization(lbm_mlp* m, float* mean_out, float* inv_std_out, float* scale_out);

/* Replace the normalisation (device float [96], [96], [3]; scales > 0), e.g.
 * to restore a trained network together with lbm_mlp_init's parameters. */
int lbm_mlp_set_normalization(lbm_mlp* m, const float* mean, const float* inv_std, const float* scale);

/* Write the network blob (lbm_closure_net_bytes bytes) for lbm_set_closure;
 * `trust` (> 0) is the largest |normalised output| accepted at run time,
 * `gain` (> 0) multiplies the correction (1 = as trained, < 1 under-relaxes
 * it), and `kmin` (>= 0) gates it by regime: the correction applies only
 * where the strip's kinetic disturbance sum |u - u_ref|^2 exceeds kmin times
 * its acoustic part sum c_s^2 (rho - rho_ref)^2 / rho0^2 (a sound wave has
 * ratio ~1, a convected vortex >> 1; 0 applies it everywhere).
 * Synchronizes the trainer's stream. */
int lbm_mlp_export(lbm_mlp* m, float trust, float gain, float kmin, void* net_out);

void lbm_mlp_destroy(lbm_mlp* m);

#ifdef __cplusplus
}
#endif

#endif /* LBM_CLOSURE_H */
