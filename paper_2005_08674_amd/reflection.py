"""Reflection measurement of a boundary condition against a larger reference.

The paper judges NSBC by eye from pressure and velocity plots (Secs. 6 and 7).
The number measured here: a test lattice and a reference lattice that is
``scale`` times larger per side start from the same analytic initial fields
(the test window centred in the reference); at every ``every``-th step the
library's fp64 energy reduction (lbm_energy) sums

    E_err(t) = sum over the window of 1/2 [c_s^2 d_rho^2 / rho0 + rho0 |d_u|^2]

of the difference test - reference.  E_0 is the same norm of the initial
disturbance measured from the uniform state (rho0, u0).  The reflection
coefficient is R_E = max_t E_err(t) / E_0 over t <= T_meas, where T_meas stops
before anything reflected at the reference's own boundary can re-enter the
window (acoustic speed c_s + |u0|).

Marshalling only: both lattices and every energy sum run on the GPU; the host
takes the maximum of the returned doubles.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import lbm as L
from .lattice import Lattice

CS = 1.0 / math.sqrt(3.0)


def fields_on(field_fn, nx: int, ny: int, x0: float = 0.0, y0: float = 0.0):
    """Evaluate field_fn(x, y) -> (drho, ux, uy) on an nx x ny lattice whose node (0, 0) sits at
    coordinate (x0, y0) of the field's frame."""
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return field_fn(x + x0, y + y0)


def clean_time(ref_nx: int, ref_ny: int, nx: int, ny: int, u0=(0.0, 0.0)) -> float:
    """Steps before a wave reflected at the reference boundary can re-enter the window."""
    d = min(ref_nx, ref_ny) / 2.0
    w = max(nx, ny) / 2.0
    return (2.0 * d - w) / (CS + math.hypot(*u0))


class ReflectionRun:
    """Test lattice plus ``scale``x reference lattice from one analytic field function."""

    def __init__(self, field_fn, nx, ny, tau, scale=4, store="f64", ref_store=None, u0=(0.0, 0.0),
                 m0=None, ubase=(0.0, 0.0), test_kw=None, ref_kw=None, rho0=1.0, closure=None):
        self.nx, self.ny, self.scale, self.u0, self.rho0 = nx, ny, scale, tuple(u0), rho0
        self.rnx, self.rny = scale * nx, scale * ny
        self.ox, self.oy = (self.rnx - nx) // 2, (self.rny - ny) // 2
        m0 = m0 if m0 is not None else (rho0, u0[0], u0[1])
        tk = dict(test_kw or {})
        rk = dict(ref_kw or {})
        self.test = Lattice(nx, ny, tau, fields_on(field_fn, nx, ny), rho0=rho0, store=store, m0=m0,
                            ubase=ubase, **tk)
        self.ref = Lattice(self.rnx, self.rny, tau, fields_on(field_fn, self.rnx, self.rny, -self.ox, -self.oy),
                           rho0=rho0, store=ref_store or store, m0=m0, ubase=ubase, **rk)
        if closure is not None:  # a network blob (lbm_mlp_export) for the test lattice's edges
            L.lbm_set_closure(self.test.ctx, closure.data_ptr(), 1)
        self.e0 = float(self.test.energy(ux_ref=u0[0], uy_ref=u0[1]).item())

    def t_clean(self) -> float:
        return clean_time(self.rnx, self.rny, self.nx, self.ny, self.u0)

    def run(self, steps: int, every: int = 5, respect_clean_time: bool = True):
        """Advance both lattices, recording E_err every ``every`` steps; returns a dict with the
        series (E_err / E_0 at t = 0, every, 2 every, ...), R_E and the measured horizon."""
        horizon = steps
        if respect_clean_time:
            horizon = min(steps, int(self.t_clean()))
        n = horizon // every + 1
        out = torch.zeros(n, dtype=torch.float64, device=self.test.device)
        base = out.data_ptr()
        for k in range(n):
            L.lbm_energy(self.test.ctx, self.ref.ctx, self.ox, self.oy, 0.0, 0.0, base + 8 * k)
            if k + 1 < n:
                self.test.step(every)
                self.ref.step(every)
        series = out.cpu().numpy() / self.e0
        return {"R_E": float(series.max()), "E0": self.e0, "series": series, "every": every,
                "horizon": (n - 1) * every, "t_clean": self.t_clean()}

    def close(self):
        self.test.close()
        self.ref.close()
