"""Pins of the oracle's multiple-relaxation-time collision (Sec. 4, eqs. mrt_lbe,
mrt_vm, mrt_rm) and of the paper's test case 1 (Sec. 6), against what the
definition and the hydrodynamic limit fix rather than against the oracle's own
formulas."""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import reflection as R
from paper_2005_08674_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
RATES = (1.9, 1.2, 1.5)   # omega_e, omega_eps, omega_q: all distinct, none equal to omega_nu below


def _velocities():
    c = np.array(json.load(open(os.path.join(GOLD, "d2q9_fig1.json")))["c"], dtype=np.float64)
    return c[:, 0], c[:, 1]


def _raw_moments():
    """The raw moments the relaxation matrix of eq. mrt_rm names, in its order:
    density, energy, energy square, j_x, q_x, j_y, q_y, p_xx, p_xy."""
    cx, cy = _velocities()
    c2 = cx * cx + cy * cy
    return np.stack([np.ones(9), c2, c2 * c2, cx, cx * c2, cy, cy * c2, cx * cx - cy * cy, cx * cy])


def test_transformation_matrix_is_the_gram_schmidt_basis():
    """Rows mutually orthogonal and span(rows 0..k) = span(raw moments 0..k) for every k: this fixes M
    up to a scale per row, which cancels in M^-1 S M."""
    M = oracle.mrt_matrix()
    raw = _raw_moments()
    G = M @ M.T
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() < 1e-13
    for k in range(9):
        coef, *_ = np.linalg.lstsq(raw[:k + 1].T, M[k], rcond=None)
        assert np.abs(raw[:k + 1].T @ coef - M[k]).max() < 1e-13, k
        assert abs(coef[k]) > 0.5, k          # the new raw moment enters each row


def _hermite_rows():
    """Closed forms of the orthogonal moments, worked out by hand from the raw moments (the usual D2Q9
    basis): e = 3|c|^2 - 4, eps = (9|c|^4 - 21|c|^2 + 8)/2, q = (3|c|^2 - 5) c, p_xx, p_xy."""
    cx, cy = _velocities()
    c2 = cx * cx + cy * cy
    return np.stack([np.ones(9), 3 * c2 - 4, (9 * c2 * c2 - 21 * c2 + 8) / 2, cx, (3 * c2 - 5) * cx,
                     cy, (3 * c2 - 5) * cy, cx * cx - cy * cy, cx * cy])


@pytest.mark.parametrize("seed", range(4))
def test_each_moment_relaxes_at_its_own_rate(seed):
    """Sec. 4: m*_k - m^eq_k = (1 - s_k)(m_k - m^eq_k), s = (C, w_e, w_eps, C, w_q, C, w_q, w_nu, w_nu);
    the conserved moments (C) are unchanged."""
    rng = np.random.default_rng(seed)
    tau = float(rng.uniform(0.5, 1.5))
    wnu = 1.0 / tau
    g = oracle.feq(1.0, 2e-3, 0.04, -0.03) + rng.normal(0, 3e-4, 9)
    m = oracle.moments_node(1.0, g)
    geq = oracle.feq(1.0, *m)
    gs = oracle.collide_node_mrt(tau, RATES, 1.0, g)
    H = _hermite_rows()
    s = np.array([0, RATES[0], RATES[1], 0, RATES[2], 0, RATES[2], wnu, wnu])
    before, after = H @ (g - geq), H @ (gs - geq)
    for k in range(9):
        assert after[k] == pytest.approx((1 - s[k]) * before[k], abs=1e-16), k


@pytest.mark.parametrize("seed", range(4))
def test_equal_rates_reduce_to_bgk(seed):
    """With every rate equal to 1/tau, M^-1 S M acts as 1/tau on the non-equilibrium part: eq. lbe_1."""
    rng = np.random.default_rng(50 + seed)
    tau = float(rng.uniform(0.51, 2.0))
    g = oracle.feq(1.0, -1e-3, 0.02, 0.05) + rng.normal(0, 1e-4, 9)
    a = oracle.collide_node_mrt(tau, (1 / tau,) * 3, 1.0, g)
    b = oracle.collide_node(tau, 1.0, g)
    assert np.abs(a - b).max() < 1e-17


def test_rates_outside_0_2_are_rejected():
    g = oracle.feq(1.0, 0.0, 0.0, 0.0)
    with pytest.raises(ValueError):
        oracle.collide_node_mrt(0.6, (2.1, 1.0, 1.0), 1.0, g)
    with pytest.raises(ValueError):
        oracle.collide_node_mrt(0.49, (1.0, 1.0, 1.0), 1.0, g)
    oracle.collide_node_mrt(0.5, (2.0, 2.0, 2.0), 1.0, g)        # tau = 1/2 is allowed for MRT
    f = W.uniform(8, 8)
    with pytest.raises(ValueError):
        oracle.Lattice(8, 8, 0.5, *f)                              # ... but not for BGK


def _shear_rate(n, tau, mrt):
    amp = 1e-4
    L = oracle.Lattice(4, n, tau, *W.shear_wave(4, n, amp), bc=(0, 0, 0, 0), mrt=mrt)
    basis = np.sin(2 * math.pi * np.arange(n) / n)

    def a():
        return float((L.moments()[1][:, 0] * basis).sum() / (basis * basis).sum())

    k = 2 * math.pi / n
    nu = (tau - 0.5) / 3
    steps = int(round(0.5 / (nu * k * k)))
    L.step(steps // 5)
    a1, t1 = a(), L.t
    L.step(steps)
    return -math.log(a() / a1) / (L.t - t1) / (nu * k * k)


def test_shear_viscosity_depends_on_omega_nu_only():
    """A shear wave decays at nu k^2 with nu = c_s^2 (1/omega_nu - 1/2), whatever the other rates are."""
    for rates in (RATES, (1.0, 1.9, 1.1)):
        r = _shear_rate(64, 0.6, rates)
        assert abs(r - 1) < 3e-3, (rates, r)


def _sound_rate(n, tau, mrt, steps):
    """Decay rate of the amplitude of a standing sound wave, from its acoustic energy (which decays at
    twice the amplitude rate), measured over `steps` steps."""
    x = np.arange(n)
    drho = np.tile(1e-5 * np.cos(2 * math.pi * x / n), (4, 1))
    z = np.zeros((4, n))
    L = oracle.Lattice(n, 4, tau, drho, z, z.copy(), bc=(0, 0, 0, 0), mrt=mrt)

    def energy():
        return R.energy(*L.moments())

    L.step(100)
    e1, t1 = energy(), L.t
    L.step(steps)
    return -math.log(energy() / e1) / (L.t - t1) / 2


@pytest.mark.parametrize("omega_e", [1.0, 1.9])
def test_sound_attenuation_gives_the_bulk_viscosity_of_omega_e(omega_e):
    """The trace of the momentum flux is the energy moment e (e = 3 tr Pi - 4 rho), so it relaxes at
    omega_e: the 2-D Navier-Stokes limit has bulk viscosity zeta = c_s^2 (1/omega_e - 1/2), and a sound
    wave's amplitude decays at (nu + zeta) k^2 / 2."""
    tau, n = 0.6, 128
    k = 2 * math.pi / n
    nu, zeta = (tau - 0.5) / 3, (1 / omega_e - 0.5) / 3
    expect = (nu + zeta) * k * k / 2
    rate = _sound_rate(n, tau, (omega_e, 1.2, 1.5), int(round(0.5 / expect)))
    assert rate == pytest.approx(expect, rel=1e-2)


def test_paper_test_case_1_plane_wave_leaves_the_domain():
    """Sec. 6, test case 1 (128^2, 60 degrees, tau = 1/2, MRT rates 1.9, gamma 0.6): the reflected energy
    left in the domain once the wave has crossed it is nearly zero, far below that of the same boundary
    without the extrapolation (gamma = 0), and the zero-viscosity run stays finite."""
    w = W.plane_wave_tc1()
    e0 = R.energy(*w.fields)
    left = {}
    for gamma in (0.6, 0.0):
        L = oracle.Lattice(w.nx, w.ny, w.tau, *w.fields, gamma=gamma, mrt=w.mrt)
        L.step(w.steps)
        assert np.isfinite(L.g).all()
        left[gamma] = R.energy(*L.moments()) / e0
    assert left[0.6] < 1e-3
    assert left[0.0] > 100 * left[0.6]
