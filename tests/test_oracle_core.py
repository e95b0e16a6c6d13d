"""Pins of the CPU oracle's bulk arithmetic (lattice, equilibrium, collision,
streaming) against facts the paper and the mathematics fix, not against the
oracle's own formulas."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2005_08674_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_lattice_matches_figure_1():
    g = json.load(open(os.path.join(GOLD, "d2q9_fig1.json")))
    cx, cy, w, opp = oracle.lattice_constants()
    assert [[int(a), int(b)] for a, b in zip(cx, cy)] == g["c"]
    for wi, s in zip(w, g["w"]):
        assert wi == pytest.approx(float(Fraction(s)), rel=1e-16)
    for i in range(9):
        assert cx[opp[i]] == -cx[i] and cy[opp[i]] == -cy[i]


def test_lattice_isotropy():
    """Weights of D2Q9 reproduce the Maxwellian's velocity moments up to 4th order with c_s^2 = 1/3."""
    cx, cy, w, _ = oracle.lattice_constants("longdouble")
    c = np.stack([cx, cy]).astype(np.longdouble)
    cs2 = np.longdouble(1) / 3
    assert abs(w.sum() - 1) < 1e-18
    assert np.all(abs(c @ w) < 1e-18)
    second = np.einsum("i,ai,bi->ab", w, c, c)
    assert np.allclose(second.astype(float), np.eye(2) / 3, atol=1e-17)
    fourth = np.einsum("i,ai,bi,ci,di->abcd", w, c, c, c, c)
    d = np.eye(2)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d))
    assert np.allclose(fourth.astype(float), float(cs2 * cs2) * iso, atol=1e-17)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moment_identities(seed):
    """The discrete equilibrium carries rho, rho u and the Euler stress rho c_s^2 I + rho u u exactly."""
    rng = np.random.default_rng(seed)
    rho0 = float(rng.uniform(0.5, 2))
    drho = float(rng.uniform(-0.1, 0.1))
    ux, uy = rng.uniform(-0.15, 0.15, size=2)
    cx, cy, w, _ = oracle.lattice_constants("longdouble")
    g = oracle.feq(rho0, drho, ux, uy, "longdouble")
    L = np.longdouble
    f = g + np.asarray(w, L) * L(rho0)
    rho, ux, uy = L(rho0) + L(drho), L(ux), L(uy)
    assert abs(g.sum() - L(drho)) < 1e-18
    assert abs((cx * f).sum() - rho * ux) < 1e-18
    assert abs((cy * f).sum() - rho * uy) < 1e-18
    pxx = (cx * cx * f).sum()
    pxy = (cx * cy * f).sum()
    pyy = (cy * cy * f).sum()
    assert abs(pxx - (rho / 3 + rho * ux * ux)) < 1e-18
    assert abs(pyy - (rho / 3 + rho * uy * uy)) < 1e-18
    assert abs(pxy - rho * ux * uy) < 1e-18
    # equilibrium at rest is w_i rho, the deviation is w_i drho
    g0 = oracle.feq(rho0, drho, 0.0, 0.0, "longdouble")
    assert np.allclose(g0.astype(float), w * drho, atol=1e-19)


@pytest.mark.parametrize("seed", range(5))
def test_collision_conserves_and_relaxes(seed):
    rng = np.random.default_rng(100 + seed)
    rho0 = 1.0
    tau = float(rng.uniform(0.51, 2.0))
    cx, cy, w, _ = oracle.lattice_constants()
    g = oracle.feq(rho0, 1e-3, 0.05, -0.02) + rng.normal(0, 1e-4, 9)
    gs = oracle.collide_node(tau, rho0, g)
    assert abs(gs.sum() - g.sum()) < 1e-17
    assert abs((cx * gs).sum() - (cx * g).sum()) < 1e-17
    assert abs((cy * gs).sum() - (cy * g).sum()) < 1e-17
    # tau = 1 lands exactly on the equilibrium of the node's own moments
    m = oracle.moments_node(rho0, g)
    assert np.allclose(oracle.collide_node(1.0, rho0, g), oracle.feq(rho0, *m), atol=1e-18)


def test_periodic_global_conservation():
    """Fully periodic lattice: total mass and momentum are invariants of collide + stream."""
    nx, ny = 48, 40
    rng = np.random.default_rng(7)
    drho = 1e-3 * rng.standard_normal((ny, nx))
    ux = 0.02 * rng.standard_normal((ny, nx))
    uy = 0.02 * rng.standard_normal((ny, nx))
    L = oracle.Lattice(nx, ny, 0.53, drho, ux, uy, bc=(0, 0, 0, 0))
    cx, cy, _, _ = oracle.lattice_constants()

    def totals():
        g = L.g
        return g.sum(), np.tensordot(cx, g, 1).sum(), np.tensordot(cy, g, 1).sum()

    m0 = totals()
    L.step(1000)
    m1 = totals()
    for a, b in zip(m0, m1):
        assert abs(a - b) < 1e-13


def _shear_rate(n, tau=0.6, steps=None):
    amp = 1e-4
    L = oracle.Lattice(4, n, tau, *W.shear_wave(4, n, amp), bc=(0, 0, 0, 0))
    basis = np.sin(2 * math.pi * np.arange(n) / n)

    def a():
        return float((L.moments()[1][:, 0] * basis).sum() / (basis * basis).sum())

    k = 2 * math.pi / n
    nu = (tau - 0.5) / 3
    steps = steps or int(round(0.5 / (nu * k * k)))
    L.step(steps // 5)
    a1, t1 = a(), L.t
    L.step(steps)
    a2, t2 = a(), L.t
    rate = -math.log(a2 / a1) / (t2 - t1)
    return rate / (nu * k * k)


def test_shear_wave_decay_and_order():
    """u_x = U sin(k y) decays as exp(-nu k^2 t), nu = (tau - 1/2)/3, with second-order convergence."""
    r32, r64, r128 = (_shear_rate(n) for n in (32, 64, 128))
    assert abs(r64 - 1) < 3e-3
    order = math.log(abs(r32 - 1) / abs(r64 - 1), 2)
    order2 = math.log(abs(r64 - 1) / abs(r128 - 1), 2)
    assert 1.8 < order < 2.2 and 1.8 < order2 < 2.2


def test_sound_speed():
    """A right-moving Gaussian plane wave travels at c_s = 1/sqrt(3) (Sec. 6)."""
    nx, ny = 1024, 4
    f = W.plane_wave(nx, ny, 0.0, 1e-4, 8.0, (256.0, 0.0))
    L = oracle.Lattice(nx, ny, 0.51, *f, bc=(0, 0, 0, 0))
    x = np.arange(nx)

    def centroid():
        d, u, v = L.moments()
        e = (d[0] ** 2 / 3 + u[0] ** 2)
        return float((x * e).sum() / e.sum())

    L.step(50)
    c1, t1 = centroid(), L.t
    L.step(550)
    c2, t2 = centroid(), L.t
    speed = (c2 - c1) / (t2 - t1)
    assert speed == pytest.approx(1 / math.sqrt(3), rel=5e-3)


def test_long_double_agrees_with_double():
    """Round-off check of the fp64 oracle: deviation form in double vs x87 extended precision."""
    w = W.pulse_128()
    a = oracle.Lattice(w.nx, w.ny, w.tau, *w.fields)
    b = oracle.Lattice(w.nx, w.ny, w.tau, *w.fields, kind="longdouble")
    for n in (10, 90, 400):
        a.step(n)
        b.step(n)
        ma, mb = a.moments(), b.moments()
        assert np.abs(ma[0] - mb[0]).max() / w.rho0 < 1e-14
        assert max(np.abs(ma[1] - mb[1]).max(), np.abs(ma[2] - mb[2]).max()) / w.u_ref < 1e-13
