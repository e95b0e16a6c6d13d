"""Oracle of the learned closure's inputs and targets (test infrastructure only).

For a boundary node b with outward unit normal n and tangent t = (-n_y, n_x),
and the far-field state m0 = (rho_ref, u_ref), the inputs are, for the strip
nodes b - d n + k t (d = 0, 1, 2; k = -1, 0, 1; node j = 3 d + k + 1 fills
inputs 9 j .. 9 j + 8):
    [rho - rho_ref, (u - u_ref).n, (u - u_ref).t, P_nn, P_nt, P_tt, Q_nnt, Q_ntt, R_nntt]
with P, Q, R the 2nd, 3rd and 4th moments of f - f^eq in the (n, t) frame
(f the post-collision populations the GPU keeps, f^eq the discrete
equilibrium of eq. feq_1 at the node's own moments); inputs 82..84 are NSBC's
m_c (eqs. nes_2, nes_3: one-sided difference along the normal at time t,
far-field blend) minus m0, as (rho, u.n, u.t).  Those 84 values are divided by
the strip amplitude A = sqrt(mean_j [c_s^2 (rho_j - rho_ref)^2 / rho0^2 +
|u_j - u_ref|^2]); input 81 is 1/tau; inputs 85, 86 are u_ref.n, u_ref.t;
87..95 are 0.  The training target of a site is (true moments at t + 1 - m_c) / A.
Computed here in fp64 from the oracle's state, straight from these
definitions.
"""
from __future__ import annotations

import numpy as np

import oracle

NORMALS = {0: (-1, 0), 1: (1, 0), 2: (0, -1), 3: (0, 1)}


def _node(post, x, y, rho0):
    """(drho, ux, uy, fneq[9]) of node (x, y) of a post-collision state."""
    g = post[:, y, x].astype(np.float64)
    cx, cy, w, _ = oracle.lattice_constants()
    drho = g.sum()
    rho = rho0 + drho
    ux, uy = (cx * g).sum() / rho, (cy * g).sum() / rho
    geq = oracle.feq(rho0, drho, ux, uy)
    return drho, ux, uy, g - geq


def site_features(lat: "oracle.Lattice", x, y, edge, gamma, beta=0.0, m0=(1.0, 0.0, 0.0), grad_order=1,
                  post=None):
    """(96 inputs, NSBC's m_c as (rho - rho0, u.n, u.t), strip amplitude A) of one site of an oracle
    lattice at its current time."""
    post = lat.post_collision() if post is None else post
    rho0 = lat.rho0
    nx_, ny_ = NORMALS[edge]
    tx, ty = -ny_, nx_
    cx, cy, _, _ = oracle.lattice_constants()
    cn = cx * nx_ + cy * ny_
    ct = cx * tx + cy * ty
    rref, uxr, uyr = m0[0] - rho0, m0[1], m0[2]
    f = np.zeros(96)
    mom = {}
    for d in range(3):
        for k in (-1, 0, 1):
            sx, sy = x - d * nx_ + k * tx, y - d * ny_ + k * ty
            drho, ux, uy, q = _node(post, sx, sy, rho0)
            j = 3 * d + k + 1
            f[9 * j:9 * j + 9] = [drho - rref, (ux - uxr) * nx_ + (uy - uyr) * ny_,
                                  (ux - uxr) * tx + (uy - uyr) * ty,
                                  (q * cn * cn).sum(), (q * cn * ct).sum(), (q * ct * ct).sum(),
                                  (q * cn * cn * ct).sum(), (q * cn * ct * ct).sum(), (q * cn * cn * ct * ct).sum()]
            if k == 0:
                mom[d] = np.array([drho, ux, uy])
    mb, m1, m2 = mom[0], mom[1], mom[2]
    dn = mb - m1 if grad_order == 1 else (3 * mb - 4 * m1 + m2) / 2
    mp = mb - gamma * dn
    ref = np.array([rref, uxr, uyr])
    mc = (1 - beta) * mp + beta * ref
    mcn = np.array([mc[0], mc[1] * nx_ + mc[2] * ny_, mc[1] * tx + mc[2] * ty])
    refn = np.array([rref, uxr * nx_ + uyr * ny_, uxr * tx + uyr * ty])
    strip = f[:81].reshape(9, 9)
    amp = np.sqrt(np.mean(strip[:, 0] ** 2 / (3.0 * rho0 ** 2) + strip[:, 1] ** 2 + strip[:, 2] ** 2))
    inv = 1.0 / amp if amp > 0 else 0.0
    f[:81] *= inv
    f[81] = 1.0 / lat.p.tau
    f[82:85] = (mcn - refn) * inv
    f[85:87] = refn[1:]
    return f, mcn, amp


def site_target(lat_next: "oracle.Lattice", x, y, edge, mcn, amp):
    """Training target of a site: (moments at t + 1 - m_c) / A, in the (n, t) frame."""
    return (site_moments(lat_next, x, y, edge) - mcn) / amp


def site_moments(lat: "oracle.Lattice", x, y, edge):
    """(rho - rho0, u.n, u.t) of node (x, y) at the lattice's current time."""
    drho, ux, uy = (m[y, x] for m in lat.moments())
    nx_, ny_ = NORMALS[edge]
    return np.array([drho, ux * nx_ + uy * ny_, -ux * ny_ + uy * nx_])
