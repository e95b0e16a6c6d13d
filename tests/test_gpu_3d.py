"""GPU D3Q19 and D3Q27 sweeps (include/lbm3d.h) against the CPU oracle of the same velocity set: fp64
storage within 1e-12 and fp32 within 1e-5 (relative, as the 2-D parity tests), every launch shape
bit-identical, periodic and NSBC face mixes, the smallest lattice."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_08674_amd import lbm
    lbm.load()


def _fields(nx, ny, nz, u0=(0.03, -0.02, 0.01), a=1e-3, w=3.0, seed=0):
    rng = np.random.default_rng(seed)
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(float)
    c = rng.uniform(0.3, 0.7, 3) * np.array([nx, ny, nz])
    dr = a * np.exp(-math.log(2) * ((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / w ** 2)
    return dr, np.full_like(dr, u0[0]), np.full_like(dr, u0[1]), np.full_like(dr, u0[2])


def _pair(nx, ny, nz, store, tol, checkpoints, bc=(1,) * 6, beta=0.3, u0=(0.03, -0.02, 0.01), tau=0.58, q=19):
    from paper_2005_08674_amd.lattice3d import Lattice3D
    print(f"\n[3d parity] D3Q{q} {nx}x{ny}x{nz} store={store} bc={bc}", flush=True)
    f = _fields(nx, ny, nz, u0)
    m0 = (1.0002, *u0)
    g = Lattice3D(nx, ny, nz, tau, f, bc=bc, store=store, beta=beta, m0=m0, q=q)
    o = oracle.Lattice3D(nx, ny, nz, tau, *f, bc=bc, beta=beta, m0=m0, q=q)
    u_ref = 0.03
    for t in checkpoints:
        g.step(t - g.t)
        o.step(t - o.t)
        gm, om = g.moments(), o.moments()
        er = np.abs(gm[0] - om[0]).max()
        eu = max(np.abs(gm[a] - om[a]).max() for a in (1, 2, 3)) / u_ref
        print(f"  t={t:4d} e_rho={er:.3e} e_u={eu:.3e}", flush=True)
        assert er <= tol and eu <= tol, (t, er, eu)
    g.close()


@pytest.mark.parametrize("dims,bc", [((20, 18, 16), (1,) * 6), ((70, 9, 11), (1, 1, 0, 0, 1, 1)),
                                     ((13, 14, 15), (0,) * 6), ((3, 3, 3), (1,) * 6), ((66, 5, 4), (0, 0, 1, 1, 0, 0))])
@pytest.mark.parametrize("q", [19, 27])
def test_fp64_against_oracle(dims, bc, q):
    _pair(*dims, "f64", 1e-12, [1, 5, 30, 80], bc=bc, q=q)


@pytest.mark.parametrize("q", [19, 27])
def test_fp32_against_oracle(q):
    _pair(40, 36, 32, "f32", 1e-5, [1, 20, 100], q=q)


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("store", ["f32", "f64", "f16", "bf16"])
def test_every_shape_bitwise_identical(store, q):
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice3d import Lattice3D
    f = _fields(70, 19, 23)
    ref = None
    ran = []
    for shape in range(lbm.lbm3d_shape_count()):
        name = lbm.lbm3d_shape_describe(shape)
        g = Lattice3D(70, 19, 23, 0.6, f, store=store, beta=0.2, m0=(1.0, 0.03, -0.02, 0.01), q=q)
        try:
            lbm.lbm3d_set_shape(g.ctx, shape)
        except lbm.LbmError:
            # the pair shapes take the 16-bit formats only
            assert name.startswith("pair") and store in ("f32", "f64"), name
            g.close()
            continue
        g.step(7)
        m = g.populations().cpu().numpy()
        g.close()
        ran.append(name)
        if ref is None:
            ref = m
        else:
            assert np.array_equal(m, ref), (store, name)
    assert any(n.startswith("pair") for n in ran) == (store in ("f16", "bf16"))


def test_pair_shapes_refuse_odd_nx_and_periodic_x():
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice3d import Lattice3D
    pair = [i for i in range(lbm.lbm3d_shape_count()) if lbm.lbm3d_shape_describe(i).startswith("pair")][0]
    g = Lattice3D(33, 16, 12, 0.6, _fields(33, 16, 12), store="f16")
    with pytest.raises(lbm.LbmError):
        lbm.lbm3d_set_shape(g.ctx, pair)
    best, times = g.autotune(reps=1)
    assert times[pair] < 0 and times[best] > 0
    g.close()
    h = Lattice3D(32, 16, 12, 0.6, _fields(32, 16, 12), store="f16", bc=(0, 0, 1, 1, 1, 1))
    with pytest.raises(lbm.LbmError):
        lbm.lbm3d_set_shape(h.ctx, pair)
    h.close()


@pytest.mark.parametrize("q", [19, 27])
def test_autotune_leaves_the_state_and_picks_a_shape(q):
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice3d import Lattice3D
    f = _fields(64, 32, 16)
    a = Lattice3D(64, 32, 16, 0.6, f, q=q)
    b = Lattice3D(64, 32, 16, 0.6, f, q=q)
    best, times = a.autotune(reps=2)
    assert 0 <= best < lbm.lbm3d_shape_count() and times[best] > 0 and a.t == 0
    names = [lbm.lbm3d_shape_describe(i) for i in range(lbm.lbm3d_shape_count())]
    assert all((t > 0) != n.startswith("pair") for t, n in zip(times, names))  # FP32: no pair shapes
    a.step(5)
    b.step(5)
    assert np.array_equal(np.array(a.moments()), np.array(b.moments()))


@pytest.mark.parametrize("store", ["f64", "f16", "bf16"])
@pytest.mark.parametrize("q", [19, 27])
def test_checkpoint_restore_continues_bitwise(q, store):
    """get_populations / set_populations round-trip the state: a lattice restored from a checkpoint
    steps on exactly as the one it was taken from (the x-face moments are rebuilt on restore; a
    16-bit value decoded and encoded again is the same value)."""
    from paper_2005_08674_amd.lattice3d import Lattice3D
    f = _fields(40, 12, 10)
    a = Lattice3D(40, 12, 10, 0.6, f, store=store, beta=0.2, m0=(1.0, 0.03, -0.02, 0.01), q=q)
    b = Lattice3D(40, 12, 10, 0.6, f, store=store, beta=0.2, m0=(1.0, 0.03, -0.02, 0.01), q=q)
    a.step(7)
    snap = a.populations()
    b.set_populations(torch.zeros_like(snap))
    b.set_populations(snap)
    assert torch.equal(b.populations(), snap)
    a.step(9)
    b.step(9)
    assert np.array_equal(np.array(a.moments()), np.array(b.moments()))
    a.close()
    b.close()


@pytest.mark.parametrize("q", [19, 27])
@pytest.mark.parametrize("bc", [(1,) * 6, (1, 1, 0, 0, 1, 1)])
def test_non_equilibrium_state_against_oracle(q, bc):
    """Start from populations away from equilibrium (f^eq plus seeded noise), set on the GPU as the
    post-collision state P.  The oracle holds the pre-collision state G whose BGK collision is P:
    G = (tau P - f^eq(m(P))) / (tau - 1), with m and f^eq from the oracle's own node functions.
    FP64 moments must agree within 1e-12 over 40 steps."""
    from paper_2005_08674_amd.lattice3d import Lattice3D
    nx, ny, nz, tau = 11, 9, 8, 0.62
    rng = np.random.default_rng(11)
    zero = np.zeros((nz, ny, nx))
    u0 = (0.02, -0.01, 0.015)
    base = [zero] + [np.full_like(zero, v) for v in u0]
    m0 = (1.0, *u0)
    g = Lattice3D(nx, ny, nz, tau, base, store="f64", bc=bc, beta=0.2, m0=m0, q=q)
    P = g.populations().cpu().numpy() + 2e-4 * rng.standard_normal((q, nz, ny, nx)) / q
    g.set_populations(P)
    o = oracle.Lattice3D(nx, ny, nz, tau, *base, bc=bc, beta=0.2, m0=m0, q=q)
    G = np.empty_like(P)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                p = P[:, z, y, x]
                geq = oracle.feq_3d(1.0, oracle.moments_node_3d(1.0, p), q=q)
                G[:, z, y, x] = (tau * p - geq) / (tau - 1)
    o.g[...] = G
    assert np.allclose(oracle.collide_node_3d(tau, 1.0, G[:, 3, 4, 5]), P[:, 3, 4, 5], atol=1e-17)
    for t in (1, 10, 40):
        g.step(t - g.t)
        o.step(t - o.t)
        gm, om = g.moments(), o.moments()
        er = np.abs(gm[0] - om[0]).max()
        eu = max(np.abs(gm[a] - om[a]).max() for a in (1, 2, 3)) / 0.02
        print(f"  D3Q{q} bc={bc} t={t} e_rho={er:.3e} e_u={eu:.3e}", flush=True)
        assert er <= 1e-12 and eu <= 1e-12, (t, er, eu)
    g.close()


def test_check_finite():
    from paper_2005_08674_amd.lattice3d import Lattice3D
    f = _fields(20, 6, 5)
    g = Lattice3D(20, 6, 5, 0.6, f, store="f32")
    g.step(3)
    assert g.check_finite()
    p = g.populations()
    p[7, 2, 3, 4] = float("nan")
    g.set_populations(p)
    assert not g.check_finite()
    g.close()


@pytest.mark.parametrize("q", [19, 27])
def test_storage_error_against_fp64(q):
    """96^3 pulses (the bench workload's recipe at a smaller size) with FP32, FP16 and BF16 storage
    (FP32 arithmetic) against the same run in FP64 (parity-checked against the oracle above) at
    t = 50 and 200: the error each format adds, relative to U_ref = c_s A_max.  Bounds as in 2-D:
    FP32 1e-5, FP16 2e-2, BF16 1e-1 (rounding of 2^-11 and 2^-8 of the stored g_i / w_i)."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd import workloads as W
    from paper_2005_08674_amd.lattice3d import Lattice3D
    n = 96
    fields, pulses = W.pulses_3d(n)
    u_ref = max(p[0] for p in pulses) / math.sqrt(3)
    runs = {s: Lattice3D(n, n, n, 0.55, fields, store=s, q=q) for s in ("f64", "f32", "f16", "bf16")}
    # at rest g_i / w_i = rho - rho0, so the FP16 exponent follows from the largest density deviation
    assert lbm.lbm3d_f16_exp(runs["f16"].ctx) == math.floor(math.log2(4096 / float(np.abs(fields[0]).max())))
    assert lbm.lbm3d_f16_exp(runs["f32"].ctx) == 0
    bounds = {"f32": 1e-5, "f16": 2e-2, "bf16": 1e-1}
    t = 0
    for t_next in (50, 200):
        for g in runs.values():
            g.step(t_next - t)
        t = t_next
        ref = runs["f64"].moments()
        for s in ("f32", "f16", "bf16"):
            m = runs[s].moments()
            er = float(np.abs(m[0] - ref[0]).max())
            eu = max(float(np.abs(m[a] - ref[a]).max()) for a in (1, 2, 3)) / u_ref
            print(f"[3d storage D3Q{q} {s} vs fp64] t={t}: e_rho={er:.3e} e_u={eu:.3e}", flush=True)
            assert er <= bounds[s] and eu <= bounds[s], (s, t, er, eu)
    for g in runs.values():
        assert g.check_finite()
        g.close()
