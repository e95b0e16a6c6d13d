"""Convenience wrapper: one D3Q19 or D3Q27 lattice on the GPU whose device memory and stream come
from PyTorch.  Marshalling only -- every computation is a call into liblbm.so (include/lbm3d.h)."""
from __future__ import annotations

import numpy as np
import torch

from . import lbm as L


class Lattice3D:
    """``fields`` = (drho, ux, uy, uz), [nz][ny][nx] arrays with drho = rho - rho0.  ``bc`` = (x low,
    x high, y low, y high, z low, z high), 1 = NSBC, 0 = periodic.  ``store`` is "f64" or "f32"; ``q`` is
    19 (D3Q19) or 27 (D3Q27)."""

    def __init__(self, nx, ny, nz, tau, fields, rho0=1.0, bc=(1,) * 6, gamma=0.6, store="f32", beta=0.0, m0=None,
                 device="cuda", stream=None, q=19):
        p = L.lbm3d_params_default()
        p.nx, p.ny, p.nz, p.tau, p.rho0, p.gamma = int(nx), int(ny), int(nz), float(tau), float(rho0), float(gamma)
        for f in range(6):
            p.bc[f] = int(bc[f])
        p.store = L.STORE_NAMES[store] if isinstance(store, str) else int(store)
        p.velocity_set = L.VELOCITY_SETS[int(q)]
        self.q = int(q)
        self.params = p
        self.shape = (int(nz), int(ny), int(nx))
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = L.lbm3d_workspace_bytes(p)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        dev = [torch.as_tensor(np.ascontiguousarray(f) if isinstance(f, np.ndarray) else f)
               .to(device=self.device, dtype=torch.float64).contiguous().reshape(self.shape) for f in fields]
        self.ctx = L.lbm3d_init(p, self.workspace.data_ptr(), nbytes, *(d.data_ptr() for d in dev),
                                self.stream.cuda_stream)
        self.stream.synchronize()
        del dev
        if m0 is not None or beta:
            self.set_farfield(beta, *(m0 if m0 is not None else (rho0, 0.0, 0.0, 0.0)))

    def set_farfield(self, beta, rho, ux, uy, uz):
        L.lbm3d_set_farfield(self.ctx, beta, rho, ux, uy, uz)

    def step(self, n: int = 1):
        L.lbm3d_step(self.ctx, n)
        return self

    @property
    def t(self) -> int:
        return L.lbm3d_time(self.ctx)

    def moments(self):
        """(rho - rho0, ux, uy, uz) as float64 numpy arrays [nz][ny][nx]."""
        out = torch.empty((4,) + self.shape, dtype=torch.float64, device=self.device)
        L.lbm3d_moments(self.ctx, out.data_ptr())
        self.stream.synchronize()
        return tuple(out.cpu().numpy())

    def populations(self):
        """The state (post-collision f_i - w_i rho0) as a float64 torch tensor [q][nz][ny][nx] on the device."""
        g = torch.empty((self.q,) + self.shape, dtype=torch.float64, device=self.device)
        L.lbm3d_get_populations(self.ctx, g.data_ptr())
        self.stream.synchronize()
        return g

    def set_populations(self, g):
        g = torch.as_tensor(g).to(device=self.device, dtype=torch.float64).contiguous()
        L.lbm3d_set_populations(self.ctx, g.data_ptr())
        self.stream.synchronize()

    def check_finite(self) -> bool:
        return L.lbm3d_check_finite(self.ctx)

    def autotune(self, reps=5):
        return L.lbm3d_autotune(self.ctx, reps)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            L.lbm3d_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
