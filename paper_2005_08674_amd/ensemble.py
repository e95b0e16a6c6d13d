"""Convenience wrapper over the ensemble C ABI (include/lbm_ensemble.h):
many independent lattices of different sizes stepped together.  Marshalling
only; the stepping, the graph capture and every kernel are in liblbm.so."""
from __future__ import annotations

import numpy as np
import torch

from . import lbm as L


def member_params(nx, ny, tau, rho0=1.0, bc=(1, 1, 1, 1), gamma=0.6, store="f32", corr_mode=0, grad_order=1,
                  corner_mode=0, ubase=(0.0, 0.0), f16_exp=None, mrt=None):
    p = L.lbm_params_default()
    p.nx, p.ny, p.tau, p.rho0, p.gamma = int(nx), int(ny), float(tau), float(rho0), float(gamma)
    for e in range(4):
        p.bc[e] = int(bc[e])
    p.store = L.STORE_NAMES[store] if isinstance(store, str) else int(store)
    p.corr_mode, p.grad_order, p.corner_mode = int(corr_mode), int(grad_order), int(corner_mode)
    p.f16_exp = L.LBM_F16_EXP_AUTO if f16_exp is None else int(f16_exp)
    p.ubase[0], p.ubase[1] = float(ubase[0]), float(ubase[1])
    if mrt is not None:
        p.collision = L.LBM_COLL_MRT
        p.omega_e, p.omega_eps, p.omega_q = (float(r) for r in mrt)
    return p


class Ensemble:
    """``members``: list of lbm_params; ``fields``: list of (drho, ux, uy) [ny][nx] arrays."""

    def __init__(self, members, fields, device="cuda", stream=None):
        self.members = list(members)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = L.lbm_ens_workspace_bytes(self.members)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        packed = [np.concatenate([np.ascontiguousarray(f[c], dtype=np.float64).ravel() for f in fields])
                  for c in range(3)]
        dev = [torch.from_numpy(a).to(self.device) for a in packed]
        self.ens = L.lbm_ens_init(self.members, self.workspace.data_ptr(), nbytes, dev[0].data_ptr(),
                                  dev[1].data_ptr(), dev[2].data_ptr(), self.stream.cuda_stream)
        del dev

    def set_farfield(self, member, beta, rho_ref, ux_ref, uy_ref):
        L.lbm_ens_set_farfield(self.ens, member, beta, rho_ref, ux_ref, uy_ref)

    def set_velocity_edge(self, member, ux, uy):
        L.lbm_ens_set_velocity_edge(self.ens, member, ux, uy)

    def step(self, n=1):
        L.lbm_ens_step(self.ens, n)

    def step_graph(self, n):
        L.lbm_ens_step_graph(self.ens, n)

    def set_log_sites(self, member_sites, twin_sites):
        """Closure training-data sites: int32 device tensors [n][4] of (member, x, y, edge) (kept alive
        here while the ensemble uses them)."""
        self._log_sites = (member_sites.contiguous(), twin_sites.contiguous())
        L.lbm_ens_set_log_sites(self.ens, self._log_sites[0].data_ptr(), self._log_sites[1].data_ptr(),
                                self._log_sites[0].shape[0])

    def step_graph_logged(self, n, log_every):
        """n steps in one graph launch, logging a record every log_every steps.  Returns float32 device
        views (feat [records][sites][96], mc [records][sites][4], resid [records][sites][3]) of the
        log buffer: record j holds the inputs at step j * log_every and the targets one step later."""
        nbytes = L.lbm_ens_log_bytes(self.ens, n, log_every)
        nsites = self._log_sites[0].shape[0]
        recs = (n + log_every - 1) // log_every
        buf = torch.empty((recs, nsites * L.LBM_ENS_LOG_FLOATS), dtype=torch.float32, device=self.device)
        assert buf.numel() * 4 == nbytes
        L.lbm_ens_step_graph(self.ens, n, buf.data_ptr(), nbytes, log_every)
        feat = buf[:, :nsites * 96].view(recs, nsites, 96)
        mc = buf[:, nsites * 96:nsites * 100].view(recs, nsites, 4)
        resid = buf[:, nsites * 100:].view(recs, nsites, 3)
        return feat, mc, resid

    @property
    def t(self):
        return L.lbm_ens_time(self.ens)

    def info(self):
        return L.lbm_ens_info(self.ens)

    def moments(self, member):
        p = self.members[member]
        out = [torch.empty((p.ny, p.nx), dtype=torch.float64, device=self.device) for _ in range(3)]
        L.lbm_ens_moments(self.ens, member, out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(), True, True)
        self.stream.synchronize()
        return tuple(o.cpu().numpy() for o in out)

    def populations(self, member):
        p = self.members[member]
        g = torch.empty((9, p.ny, p.nx), dtype=torch.float64, device=self.device)
        L.lbm_ens_get_populations(self.ens, member, g.data_ptr())
        self.stream.synchronize()
        return g.cpu().numpy()

    def autotune(self, reps=5):
        return L.lbm_ens_autotune(self.ens, reps)

    def set_two_step(self, shape_id):
        """Two-step sweep shape (-1: single steps)."""
        L.lbm_ens_set_two_step(self.ens, shape_id)

    def autotune_two_step(self, reps=5):
        return L.lbm_ens_autotune_two_step(self.ens, reps)

    def close(self):
        if getattr(self, "ens", None) is not None:
            L.lbm_ens_destroy(self.ens)
            self.ens = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
