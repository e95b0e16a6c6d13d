"""Convenience wrapper: one GPU lattice whose device memory and stream come
from PyTorch.  Marshalling only -- every computation is a call into liblbm.so
through ``paper_2005_08674_amd.lbm``."""
from __future__ import annotations

import numpy as np
import torch

from . import lbm as L


class Lattice:
    """D2Q9 lattice (BGK, or MRT with ``mrt`` = (omega_e, omega_eps, omega_q)) with NSBC/periodic
    edges on one GPU.  Edges: 1 = NSBC, 0 = periodic, 2 = Dirichlet velocity at ``uw`` (left/right
    with periodic bottom/top).

    ``fields`` = (drho, ux, uy), [ny][nx] arrays (numpy or torch) with
    drho = rho - rho0.  ``bc`` = (left, right, bottom, top), 1 = NSBC,
    0 = periodic.  ``store`` is "f64", "f32", "f16" or "bf16".  ``ubase`` is the base
    velocity u_b of the stored deviations f_i - f^eq_i(rho0, u_b).
    """

    def __init__(self, nx, ny, tau, fields, rho0=1.0, bc=(1, 1, 1, 1), gamma=0.6, store="f32",
                 beta=0.0, m0=None, corr_mode=0, grad_order=1, corner_mode=0, f16_exp=None,
                 ubase=(0.0, 0.0), mrt=None, uw=None, device="cuda", stream=None):
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
        self.params = p
        self.nx, self.ny, self.rho0 = int(nx), int(ny), float(rho0)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = L.lbm_workspace_bytes(p)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        dev = [torch.as_tensor(np.ascontiguousarray(f) if isinstance(f, np.ndarray) else f)
               .to(device=self.device, dtype=torch.float64).contiguous().reshape(ny, nx) for f in fields]
        self.ctx = L.lbm_init(p, self.workspace.data_ptr(), nbytes, dev[0].data_ptr(), dev[1].data_ptr(),
                              dev[2].data_ptr(), self.stream.cuda_stream)
        del dev
        if m0 is not None:
            self.set_farfield(beta, *m0)
        elif beta:
            self.set_farfield(beta, rho0, 0.0, 0.0)
        if uw is not None:
            L.lbm_set_velocity_edge(self.ctx, *uw)

    # --------------------------------------------------------------- calls
    def set_farfield(self, beta, rho_ref, ux_ref, uy_ref):
        L.lbm_set_farfield(self.ctx, beta, rho_ref, ux_ref, uy_ref)

    def step(self, n: int = 1):
        L.lbm_step(self.ctx, n)
        return self

    @property
    def t(self) -> int:
        return L.lbm_time(self.ctx)

    def moments(self, f64: bool = True, deviation: bool = True):
        """(rho - rho0, ux, uy) as device tensors [ny][nx] (synchronised)."""
        dt = torch.float64 if f64 else torch.float32
        out = [torch.empty((self.ny, self.nx), dtype=dt, device=self.device) for _ in range(3)]
        L.lbm_moments(self.ctx, out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(), f64, deviation)
        self.stream.synchronize()
        return tuple(out)

    def moments_np(self):
        return tuple(t.cpu().numpy() for t in self.moments())

    def populations(self):
        g = torch.empty((9, self.ny, self.nx), dtype=torch.float64, device=self.device)
        L.lbm_get_populations(self.ctx, g.data_ptr())
        self.stream.synchronize()
        return g

    def set_populations(self, g):
        g = torch.as_tensor(g).to(device=self.device, dtype=torch.float64).contiguous()
        L.lbm_set_populations(self.ctx, g.data_ptr())
        self.stream.synchronize()

    def save(self) -> bytes:
        """Checkpoint (header + populations as stored) as host bytes (lbm_save)."""
        return L.lbm_save(self.ctx)

    def load(self, data: bytes):
        """Restore a checkpoint taken on a lattice with the same parameters (lbm_load)."""
        L.lbm_load(self.ctx, data)

    def check_finite(self) -> bool:
        return L.lbm_check_finite(self.ctx)

    def energy(self, ref=None, x_off=0, y_off=0, ux_ref=0.0, uy_ref=0.0, out=None):
        """fp64 acoustic energy of (self - ref window) or of (self - uniform state)."""
        if out is None:
            out = torch.zeros(1, dtype=torch.float64, device=self.device)
        L.lbm_energy(self.ctx, ref.ctx if ref is not None else None, x_off, y_off, ux_ref, uy_ref, out.data_ptr())
        return out

    def autotune(self, reps=5):
        return L.lbm_autotune(self.ctx, reps)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            L.lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
