"""Seeded synthetic inputs: initial macroscopic fields and lattice parameters.

This module draws random numbers and evaluates the analytic initial fields of
the paper's test cases; it holds none of the lattice-Boltzmann arithmetic and
imports neither the GPU library nor the oracle, so both sides can take their
inputs from it.

All fields are float64 arrays of shape [ny][nx] (x fastest); node (x, y) sits
at integer coordinates, x in [0, nx-1], y in [0, ny-1].  Density is returned as
the deviation drho = rho - rho0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

CS = 1.0 / math.sqrt(3.0)  # lattice speed of sound (Sec. 3)
NSBC_ALL = (1, 1, 1, 1)    # (left, right, bottom, top), 1 = NSBC, 0 = periodic, 2 = Dirichlet velocity


def _grid(nx: int, ny: int):
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return x, y


def gaussian_pulses_xy(x, y, pulses: Sequence[Tuple[float, float, float, float]], u0=(0.0, 0.0)):
    """Superposed Gaussian density pulses on a uniform flow, at coordinates (x, y).

    Each pulse is (amplitude A, half-width at half-maximum w, x_c, y_c):
    drho = sum A exp(-ln2 d^2 / w^2), u = u0 everywhere.
    """
    drho = np.zeros(np.shape(x))
    for a, w, xc, yc in pulses:
        d2 = (x - xc) ** 2 + (y - yc) ** 2
        drho += a * np.exp(-math.log(2.0) * d2 / (w * w))
    return drho, np.full(np.shape(x), float(u0[0])), np.full(np.shape(x), float(u0[1]))


def gaussian_pulses(nx: int, ny: int, pulses: Sequence[Tuple[float, float, float, float]],
                    u0: Tuple[float, float] = (0.0, 0.0)):
    """gaussian_pulses_xy on the nx x ny lattice."""
    x, y = _grid(nx, ny)
    return gaussian_pulses_xy(x, y, pulses, u0)


def lamb_oseen_xy(x, y, x0: float, y0: float, rc: float, uv: float, u0=(0.1, 0.0), rho0: float = 1.0):
    """Lamb-Oseen vortex on a uniform flow (Sec. 7, eqs. cv_u, cv_v, cv_d), at coordinates (x, y).

    With d^2 = (x-x0)^2 + (y-y0)^2 and the swirl amplitude U_v = beta*u0:
      u = u0x - U_v (y-y0)/R_c exp(-d^2/(2 R_c^2))
      v = u0y + U_v (x-x0)/R_c exp(-d^2/(2 R_c^2))
      rho = rho0 (1 - U_v^2/(2 C_v) exp(-d^2/R_c^2)),  C_v = c_s^2 in 2-D, exponent 1/(gamma-1) = 1.
    The swirl speed peaks at d = R_c with value U_v e^{-1/2}.
    """
    d2 = (x - x0) ** 2 + (y - y0) ** 2
    e = np.exp(-d2 / (2.0 * rc * rc))
    ux = u0[0] - uv * (y - y0) / rc * e
    uy = u0[1] + uv * (x - x0) / rc * e
    drho = -rho0 * uv * uv / (2.0 * CS * CS) * e * e
    return drho, ux, uy


def lamb_oseen(nx: int, ny: int, x0: float, y0: float, rc: float, uv: float,
               u0: Tuple[float, float] = (0.1, 0.0), rho0: float = 1.0, offset=(0.0, 0.0)):
    """lamb_oseen_xy on the nx x ny lattice; ``offset`` shifts the lattice coordinates."""
    x, y = _grid(nx, ny)
    return lamb_oseen_xy(x + offset[0], y + offset[1], x0, y0, rc, uv, u0, rho0)


def swirl_amplitude(max_swirl: float) -> float:
    """U_v such that the peak swirl speed U_v e^{-1/2} equals ``max_swirl``."""
    return max_swirl * math.exp(0.5)


def plane_wave(nx: int, ny: int, theta: float, zeta: float, lam: float,
               center: Tuple[float, float], rho0: float = 1.0):
    """Gaussian plane acoustic wave travelling along +(cos theta, sin theta) (Sec. 6, eqs. pw_p..pw_s).

    xi = (x - x_c) cos theta + (y - y_c) sin theta,
    s = sqrt(e) zeta / (rho0 lam) xi exp(-xi^2 / (2 lam^2)),  rho = rho0 (1 + s),  u = c_s s (cos, sin).
    """
    x, y = _grid(nx, ny)
    xi = (x - center[0]) * math.cos(theta) + (y - center[1]) * math.sin(theta)
    s = math.sqrt(math.e) * zeta / (rho0 * lam) * xi * np.exp(-xi * xi / (2.0 * lam * lam))
    return rho0 * s, CS * s * math.cos(theta), CS * s * math.sin(theta)


def shear_wave(nx: int, ny: int, amp: float):
    """u_x = amp sin(2 pi y / ny), u_y = 0, uniform density."""
    _, y = _grid(nx, ny)
    return np.zeros((ny, nx)), amp * np.sin(2.0 * math.pi * y / ny), np.zeros((ny, nx))


def uniform(nx: int, ny: int, drho: float = 0.0, u0=(0.0, 0.0)):
    return (np.full((ny, nx), float(drho)), np.full((ny, nx), float(u0[0])),
            np.full((ny, nx), float(u0[1])))


# --------------------------------------------------------------------------
# Named workloads.  Each returns a dict of lattice parameters plus the fields.
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    tau: float
    steps: int
    fields: Tuple[np.ndarray, np.ndarray, np.ndarray]
    rho0: float = 1.0
    bc: Tuple[int, int, int, int] = NSBC_ALL
    gamma: float = 0.6
    beta: float = 0.0
    m0: Tuple[float, float, float] = (1.0, 0.0, 0.0)
    u_ref: float = 0.0            # velocity scale for relative velocity errors
    extra: dict = field(default_factory=dict)
    mrt: Tuple[float, float, float] = None   # (omega_e, omega_eps, omega_q) for the MRT collision, else BGK
    uw: Tuple[float, float] = (0.0, 0.0)     # velocity of Dirichlet velocity edges


def pulse_128(nx: int = 128, ny: int = 128) -> Workload:
    """128x128, tau 0.6, one centred pulse A = 1e-3, HWHM 6; 1000 steps (the fp64 parity case)."""
    a, w = 1e-3, 6.0
    f = gaussian_pulses(nx, ny, [(a, w, (nx - 1) / 2.0, (ny - 1) / 2.0)])
    return Workload("pulse128_f64", nx, ny, 0.6, 1000, f, u_ref=CS * a)


def plane_wave_tc1(n: int = 128, theta_deg: float = 60.0) -> Workload:
    """Test case 1 of Sec. 6: n x n (128^2), NSBC on all edges (gamma 0.6, beta 0), a Gaussian plane
    wave (rho0 1, zeta 0.01, lambda = n/32) through the centre travelling at 60 degrees to the x axis;
    tau = 1/2 (zero shear viscosity) with the MRT rates omega_e = omega_eps = omega_q = 1.9."""
    zeta, lam = 0.01, n / 32.0
    th = math.radians(theta_deg)
    f = plane_wave(n, n, th, zeta, lam, ((n - 1) / 2.0, (n - 1) / 2.0))
    return Workload(f"planewave{n}_tc1", n, n, 0.5, 400, f, u_ref=CS * zeta, mrt=(1.9, 1.9, 1.9),
                    extra={"theta": th, "zeta": zeta, "lam": lam})


def convected_vortex_tc2(n: int = 128, nx: int = None) -> Workload:
    """Test case 2 of Sec. 7: n x n (128^2), a Dirichlet velocity inlet u_w = (u0, 0) on the left, NSBC
    (gamma 0.6, beta 0, m0 = (1, u0, 0)) on the right, periodic bottom and top; Lamb-Oseen vortex with
    u0 = 0.1, U_v = beta u0 = 0.05, R_c = 20 centred in the n x n window; Re = u0 n / nu = 1000, so
    tau = 1/2 + 3 u0 n / 1000; MRT rates omega_e = omega_eps = 1.4, omega_q = 1.2.  `nx` widens the lattice
    to the right (a reference for the window [0, n) x [0, n))."""
    u0, uv, rc = 0.1, 0.05, 20.0
    nx = nx or n
    c = (n - 1) / 2.0
    f = lamb_oseen(nx, n, c, c, rc, uv, (u0, 0.0))
    return Workload(f"convectedvortex{n}_tc2", nx, n, 0.5 + 3.0 * u0 * n / 1000.0, 2000, f, bc=(2, 1, 0, 0),
                    m0=(1.0, u0, 0.0), u_ref=u0, mrt=(1.4, 1.4, 1.2), uw=(u0, 0.0),
                    extra={"x0": c, "y0": c, "rc": rc, "uv": uv})


def vortex_512x256(seed: int = 2, nx: int = 512, ny: int = 256) -> Workload:
    """512x256, tau 0.55, inflow (0.1, 0), Lamb-Oseen R_c = 12, max swirl 0.02 at a seeded position."""
    rng = np.random.default_rng(seed)
    x0, y0 = rng.uniform(96, 160, size=2)
    y0 = y0 * ny / 256.0
    uv = swirl_amplitude(0.02)
    f = lamb_oseen(nx, ny, x0, y0, 12.0, uv, (0.1, 0.0))
    return Workload("vortex512x256_f32", nx, ny, 0.55, 5000, f, m0=(1.0, 0.1, 0.0), u_ref=0.1,
                    extra={"x0": x0, "y0": y0, "rc": 12.0, "uv": uv})


def pulses_4096(seed: int = 3, n: int = 4096) -> Workload:
    """n x n (4096^2 by default), tau 0.51, 8 seeded pulses A ~ U[1e-4,1e-3], HWHM ~ U[4,16]."""
    rng = np.random.default_rng(seed)
    lo, hi = n / 16.0, n - n / 16.0
    pulses = [(rng.uniform(1e-4, 1e-3), rng.uniform(4, 16), rng.uniform(lo, hi), rng.uniform(lo, hi))
              for _ in range(8)]
    f = gaussian_pulses(n, n, pulses)
    amax = max(p[0] for p in pulses)
    return Workload(f"pulses{n}", n, n, 0.51, 2000, f, u_ref=CS * amax, extra={"pulses": pulses})


def vortex_pulse_2048(seed: int = 5, n: int = 2048) -> Workload:
    """n x n (2048^2), tau 0.55, u0 = (0.1, 0); vortex (R_c 12, max swirl 0.02) near (3n/4, n/2) plus a
    centred pulse A = 1e-3, HWHM 8."""
    rng = np.random.default_rng(seed)
    jx, jy = rng.uniform(-32, 32, size=2) * n / 2048.0
    x0, y0 = 0.75 * n + jx, 0.5 * n + jy
    uv = swirl_amplitude(0.02)
    dv, ux, uy = lamb_oseen(n, n, x0, y0, 12.0, uv, (0.1, 0.0))
    dp, _, _ = gaussian_pulses(n, n, [(1e-3, 8.0, n / 2.0, n / 2.0)])
    return Workload(f"vortexpulse{n}", n, n, 0.55, 6000, (dv + dp, ux, uy), m0=(1.0, 0.1, 0.0),
                    u_ref=0.1, extra={"x0": x0, "y0": y0, "rc": 12.0, "uv": uv})


def pulses_3d(n: int = 256, seed: int = 6, count: int = 8):
    """n^3 D3Q19 workload: `count` seeded Gaussian pulses (A ~ U[1e-4, 1e-3], HWHM ~ U[4, 16], centres
    ~ U[n/16, 15n/16]^3) at rest; returns (fields, pulses) with fields [nz][ny][nx] (drho, ux, uy, uz)."""
    rng = np.random.default_rng(seed)
    lo, hi = n / 16.0, n - n / 16.0
    pulses = [(rng.uniform(1e-4, 1e-3), rng.uniform(4, 16), *rng.uniform(lo, hi, 3)) for _ in range(count)]
    z, y, x = np.mgrid[0:n, 0:n, 0:n].astype(np.float32)
    dr = np.zeros((n, n, n), np.float64)
    for a, w, cx, cy, cz in pulses:
        dr += a * np.exp(-math.log(2.0) * ((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) / (w * w))
    zero = np.zeros_like(dr)
    return (dr, zero, zero.copy(), zero.copy()), pulses


@dataclass
class EnsembleMember:
    nx: int
    ny: int
    tau: float
    kind: str                    # "pulse" or "vortex"
    params: dict


def ensemble_members(count: int = 256, seed: int = 4, lo: int = 64, hi: int = 512) -> List[EnsembleMember]:
    """Uneven lattices: N_x, N_y ~ U{lo..hi}, tau ~ U[0.52, 0.8], pulse or vortex with p = 1/2."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        nx, ny = (int(v) for v in rng.integers(lo, hi + 1, size=2))
        tau = float(rng.uniform(0.52, 0.8))
        if rng.uniform() < 0.5:
            a = float(rng.uniform(1e-4, 1e-3))
            w = float(rng.uniform(4, 16))
            xc = float(rng.uniform(nx / 4, 3 * nx / 4))
            yc = float(rng.uniform(ny / 4, 3 * ny / 4))
            out.append(EnsembleMember(nx, ny, tau, "pulse", {"a": a, "w": w, "xc": xc, "yc": yc}))
        else:
            speed = float(rng.uniform(0.05, 0.1))
            ang = float(rng.uniform(0, 2 * math.pi))
            swirl = float(rng.uniform(0.005, 0.02))
            rc = float(rng.uniform(4, 12))
            xc = float(rng.uniform(nx / 4, 3 * nx / 4))
            yc = float(rng.uniform(ny / 4, 3 * ny / 4))
            out.append(EnsembleMember(nx, ny, tau, "vortex",
                                      {"u0": (speed * math.cos(ang), speed * math.sin(ang)),
                                       "uv": swirl_amplitude(swirl), "rc": rc, "xc": xc, "yc": yc}))
    return out


def member_fields(m: EnsembleMember, offset=(0.0, 0.0), nx=None, ny=None):
    """Initial fields of an ensemble member; ``offset``/``nx``/``ny`` evaluate the same analytic
    field on a larger lattice whose node (offset) coincides with the member's node (0, 0)."""
    nx = m.nx if nx is None else nx
    ny = m.ny if ny is None else ny
    p = m.params
    if m.kind == "pulse":
        return gaussian_pulses(nx, ny, [(p["a"], p["w"], p["xc"] + offset[0], p["yc"] + offset[1])])
    return lamb_oseen(nx, ny, p["xc"] + offset[0], p["yc"] + offset[1], p["rc"], p["uv"], p["u0"])


def member_m0(m: EnsembleMember):
    if m.kind == "pulse":
        return (1.0, 0.0, 0.0)
    return (1.0, m.params["u0"][0], m.params["u0"][1])
