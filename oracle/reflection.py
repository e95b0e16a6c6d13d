"""FP64 reflection-energy norm (test infrastructure only).

The paper judges its boundary by eye from pressure and velocity plots (the
figures of Secs. 6 and 7).  The number used here: the acoustic energy density
of a perturbation (drho, du) about a state of density rho0,
    e = 1/2 [ c_s^2 drho^2 / rho0 + rho0 |du|^2 ],
summed over a window W.  The reflection energy at time t is the sum over W of
e for the difference between a test lattice and a reference lattice that is
larger on every side (so nothing it reflects reaches W during the
measurement); E_0 is the same sum for the initial disturbance measured from
the uniform state.  R_E = max_t E_err(t) / E_0.
"""
from __future__ import annotations

import numpy as np

CS2 = 1.0 / 3.0


def energy(drho, ux, uy, rho0: float = 1.0) -> float:
    """Sum over all given nodes of 1/2 [c_s^2 drho^2/rho0 + rho0 (ux^2 + uy^2)], in fp64."""
    drho = np.asarray(drho, np.float64)
    ux = np.asarray(ux, np.float64)
    uy = np.asarray(uy, np.float64)
    e = 0.5 * (CS2 * drho * drho / rho0 + rho0 * (ux * ux + uy * uy))
    return float(np.sum(e, dtype=np.float64))


def energy_diff(test, ref_window, rho0: float = 1.0) -> float:
    """Energy of (test - reference) where both are (drho, ux, uy) tuples over the same window."""
    return energy(test[0] - ref_window[0], test[1] - ref_window[1], test[2] - ref_window[2], rho0)


def window(fields, x0: int, y0: int, nx: int, ny: int):
    """Cut the [ny][nx] window whose lower-left node is (x0, y0) from each field."""
    return tuple(np.asarray(f)[y0:y0 + ny, x0:x0 + nx] for f in fields)


def clean_time(ref_half: float, win_half: float, u0: float = 0.0) -> float:
    """Steps before a wave reflected at the reference's own boundary can re-enter the window:
    it travels ref_half out and ref_half - win_half back at speed c_s + |u0|."""
    return (2.0 * ref_half - win_half) / (np.sqrt(CS2) + abs(u0))
