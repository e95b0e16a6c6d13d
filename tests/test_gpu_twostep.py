"""GPU multi-step sweeps: one launch advancing t -> t + 2 (level t + 1 in LDS)
or t -> t + 3 (levels t + 1 and t + 2 in LDS) must give the same bits as single
steps, for every shape, storage format, NSBC reading and ragged size, and agree
with the oracle at full size."""
import numpy as np
import pytest

import oracle
from paper_2005_08674_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_08674_amd import lbm
    lbm.load()


def _pair(nx, ny, store, shape, steps, **kw):
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    rng = np.random.default_rng(nx * 1000 + ny)
    f = W.gaussian_pulses(nx, ny, [(8e-4, max(2.0, min(nx, ny) / 6), rng.uniform(0, nx), rng.uniform(0, ny))],
                          u0=kw.pop("u0", (0.03, -0.02)))
    m0 = kw.pop("m0", (1.0002, 0.03, -0.02))
    beta = kw.pop("beta", 0.2)
    a = Lattice(nx, ny, 0.57, f, store=store, beta=beta, m0=m0, **kw)
    b = Lattice(nx, ny, 0.57, f, store=store, beta=beta, m0=m0, **kw)
    lbm.lbm_set_two_step(b.ctx, shape)
    a.step(steps)
    b.step(steps)
    pa, pb = a.populations().cpu().numpy(), b.populations().cpu().numpy()
    a.close()
    b.close()
    return pa, pb


SIZES = [(203, 77), (61, 5), (3, 3), (4, 3), (3, 40), (62, 64), (121, 130), (240, 33), (241, 129), (480, 257)]


def _three_step_takes(name, store, nx, ny):
    """Whether three-step shape `name` ("3step:64xTY/...") runs on an nx x ny lattice in `store`:
    whole tiles, and the two LDS levels (9 x ((TY + 4) x 68 + (TY + 2) x 66) stored values) within
    160 KiB."""
    ty = int(name.split("x")[1].split("/")[0])
    return nx >= 64 and ny >= ty and three_step_lds_fits(store, ty)


def three_step_lds_fits(store, ty):
    es = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[store]
    return 9 * ((ty + 4) * 68 + (ty + 2) * 66) * es <= 160 * 1024


@pytest.mark.parametrize("store", ["f64", "f32", "f16", "bf16"])
def test_bitwise_equal_to_single_steps_all_shapes(store):
    """9 steps (two-step: 4 launches and a single step) or 11 (three-step: 3 launches and 2 single
    steps); three-step shapes refuse exactly the lattices they cannot take."""
    from paper_2005_08674_amd import lbm
    for shape in range(lbm.lbm_two_step_count()):
        name = lbm.lbm_two_step_describe(shape)
        k = lbm.lbm_two_step_steps(shape)
        for nx, ny in SIZES:
            print(f"[multi-step] {store} {name} {nx}x{ny}", flush=True)
            if k == 3 and not _three_step_takes(name, store, nx, ny):
                with pytest.raises(lbm.LbmError):
                    _pair(nx, ny, store, shape, 11)
                continue
            pa, pb = _pair(nx, ny, store, shape, 9 if k == 2 else 11)
            assert np.isfinite(pa).all()
            assert np.array_equal(pa, pb), (store, name, nx, ny, np.argwhere(pa != pb)[:5])


@pytest.mark.parametrize("kw", [dict(grad_order=2), dict(corner_mode=1), dict(corr_mode=1),
                                dict(ubase=(0.03, -0.02)), dict(gamma=0.3, beta=0.0)])
def test_bitwise_equal_nsbc_readings(kw):
    from paper_2005_08674_amd import lbm
    three = [k for k in range(lbm.lbm_two_step_count()) if lbm.lbm_two_step_steps(k) == 3]
    for nx, ny in [(130, 67), (64, 3)]:
        print(f"[two-step] {kw} {nx}x{ny}", flush=True)
        pa, pb = _pair(nx, ny, "f32", 1, 12, **dict(kw))
        assert np.array_equal(pa, pb), (kw, nx, ny)
    for nx, ny in [(130, 67), (64, 12)]:
        print(f"[three-step] {kw} {nx}x{ny}", flush=True)
        pa, pb = _pair(nx, ny, "f32", three[0], 13, **dict(kw))
        assert np.array_equal(pa, pb), (kw, nx, ny)


def test_unsupported_lattices_are_refused():
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    f = W.uniform(40, 30)
    p = Lattice(40, 30, 0.6, f, store="f32", bc=(0, 0, 1, 1))
    with pytest.raises(lbm.LbmError):
        lbm.lbm_set_two_step(p.ctx, 0)
    d = Lattice(40, 30, 0.6, f, store="f64")
    lbm.lbm_set_two_step(d.ctx, 0)
    with pytest.raises(lbm.LbmError):
        lbm.lbm_set_two_step(d.ctx, lbm.lbm_two_step_count())
    lbm.lbm_set_two_step(d.ctx, -1)


def test_timing_counts_launches_and_odd_steps():
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    f = W.gaussian_pulses(100, 90, [(1e-3, 5.0, 50.0, 45.0)])
    g = Lattice(100, 90, 0.6, f, store="f32")
    lbm.lbm_set_two_step(g.ctx, 1)
    lbm.lbm_enable_timing(g.ctx, True)
    g.step(7)
    ms, n = lbm.lbm_two_step_times(g.ctx)
    bm, bn, em, en = lbm.lbm_kernel_times(g.ctx)
    assert n == 3 and bn == 1 and en == 0 and ms > 0  # the odd step is one fused launch
    assert g.t == 7


@pytest.mark.parametrize("store", ["f32", "f16"])
def test_autotuners_leave_the_state_and_time(store):
    """Both tuners time consecutive steps from a saved state: afterwards the populations and t are
    what they were, and stepping on gives the bits of an untuned twin."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    f = W.gaussian_pulses(200, 150, [(1e-3, 9.0, 90.0, 70.0)], u0=(0.02, 0.01))
    a = Lattice(200, 150, 0.58, f, store=store, m0=(1.0, 0.02, 0.01), beta=0.1)
    b = Lattice(200, 150, 0.58, f, store=store, m0=(1.0, 0.02, 0.01), beta=0.1)
    a.step(5)
    b.step(5)
    before = a.populations().cpu().numpy()
    best, times = lbm.lbm_autotune(a.ctx, 2)
    b2, t2 = lbm.lbm_autotune_two_step(a.ctx, 2)
    assert a.t == 5 and np.array_equal(a.populations().cpu().numpy(), before)
    assert times[best] > 0 and t2[b2] > 0 and lbm.lbm_get_two_step(a.ctx) == b2
    a.step(7)
    b.step(7)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())
    a.close()
    b.close()


def test_closure_falls_back_to_single_steps():
    """With the closure active the two-step shape is ignored: same bits as the closure alone."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.closure import Trainer, pack_params
    from paper_2005_08674_amd.lattice import Lattice
    p = {"W1": np.zeros((64, 96)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
         "W3": np.zeros((3, 64)), "b3": np.array([0.01, 0.02, -0.01])}
    tr = Trainer(pack_params(p), max_batch=1024)
    blob = tr.export(4.0)
    f = W.lamb_oseen(90, 70, 40.0, 30.0, 5.0, 0.03, (0.05, 0.0))
    a = Lattice(90, 70, 0.6, f, store="f32", m0=(1.0, 0.05, 0.0))
    b = Lattice(90, 70, 0.6, f, store="f32", m0=(1.0, 0.05, 0.0))
    lbm.lbm_set_closure(a.ctx, blob.data_ptr(), 1)
    lbm.lbm_set_closure(b.ctx, blob.data_ptr(), 1)
    lbm.lbm_set_two_step(b.ctx, 0)
    a.step(10)
    b.step(10)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())


def test_remainder_of_two_after_three_step_launches():
    """After three-step launches a remainder of two steps runs as one two-step launch, any other
    remainder as single steps: n = 1, 2, 4, 5 give the bits and the time of n single steps, and the
    timing counts the launches that ran."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    three = [k for k in range(lbm.lbm_two_step_count()) if lbm.lbm_two_step_steps(k) == 3
             and "64x12/768" in lbm.lbm_two_step_describe(k)][0]
    f = W.gaussian_pulses(203, 77, [(1e-3, 6.0, 70.0, 40.0)], u0=(0.02, -0.01))
    for store in ("f32", "f64", "f16"):
        a = Lattice(203, 77, 0.57, f, store=store, beta=0.2, m0=(1.0002, 0.02, -0.01))
        b = Lattice(203, 77, 0.57, f, store=store, beta=0.2, m0=(1.0002, 0.02, -0.01))
        lbm.lbm_set_two_step(b.ctx, three)
        for n, (multi, single) in zip((1, 2, 4, 5), ((0, 1), (1, 0), (1, 1), (2, 0))):
            print(f"[remainder] {store} n={n}", flush=True)
            lbm.lbm_enable_timing(b.ctx, True)
            a.step(n)
            b.step(n)
            ms, nm = lbm.lbm_two_step_times(b.ctx)
            bm, bn, em, en = lbm.lbm_kernel_times(b.ctx)
            lbm.lbm_enable_timing(b.ctx, False)
            assert (nm, bn) == (multi, single), (store, n, nm, bn)
            assert a.t == b.t
            assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy()), (store, n)
        a.close()
        b.close()


@pytest.mark.parametrize("store", ["f64", "f32", "f16", "bf16"])
def test_march_shapes_on_many_strips_and_chunks(store):
    """Every column-march shape (two- and three-step) on a 1000 x 999 lattice: 14 strips of 8 to 11
    chunks each (a shorter last chunk) beside the edge tiles; 11 steps (three-step: 3 launches and a
    two-step remainder; two-step: 5 launches and a single step) give the bits of 11 single steps."""
    from paper_2005_08674_amd import lbm
    march = [k for k in range(lbm.lbm_two_step_count()) if "+march" in lbm.lbm_two_step_describe(k)]
    assert len(march) >= 4
    for shape in march:
        name = lbm.lbm_two_step_describe(shape)
        print(f"[march] {store} {name} 1000x999", flush=True)
        if lbm.lbm_two_step_steps(shape) == 3 and not _three_step_takes(name, store, 1000, 999):
            with pytest.raises(lbm.LbmError):
                _pair(1000, 999, store, shape, 11)
            continue
        pa, pb = _pair(1000, 999, store, shape, 11)
        assert np.isfinite(pa).all()
        assert np.array_equal(pa, pb), (store, name, np.argwhere(pa != pb)[:5])


def test_full_size_4096_tuned_launch_against_single_and_oracle():
    """4096^2 FP32 (the HBM workload) in the launch the benchmark times (the autotuner's cached choice,
    three steps per launch): 99 steps (33 launches) bit-identical to the single-step path and within
    the FP32 bound of the oracle at t = 99."""
    from paper_2005_08674_amd import autotune, lbm
    from paper_2005_08674_amd.lattice import Lattice
    w = W.pulses_4096()
    a = Lattice(w.nx, w.ny, w.tau, w.fields, store="f32")
    name = autotune.apply(a, "f32")
    if name is None:
        autotune.tune(a, "f32", reps=3, path=None)
    shape = lbm.lbm_get_two_step(a.ctx)
    print(f"\n[4096^2 tuned] {name} -> multi-step shape {lbm.lbm_two_step_describe(shape) if shape >= 0 else None}",
          flush=True)
    lbm.lbm_enable_timing(a.ctx, True)
    a.step(99)
    ms, launches = lbm.lbm_two_step_times(a.ctx)
    lbm.lbm_enable_timing(a.ctx, False)
    if shape >= 0:
        assert launches == 99 // lbm.lbm_two_step_steps(shape)
    ga = a.populations().cpu().numpy()
    gm = a.moments_np()
    a.close()
    b = Lattice(w.nx, w.ny, w.tau, w.fields, store="f32")
    b.step(99)
    assert np.array_equal(ga, b.populations().cpu().numpy())
    b.close()
    del ga
    o = oracle.Lattice(w.nx, w.ny, w.tau, *w.fields)
    o.step(99)
    om = o.moments()
    er = np.abs(gm[0] - om[0]).max()
    eu = max(np.abs(gm[1] - om[1]).max(), np.abs(gm[2] - om[2]).max()) / w.u_ref
    print(f"[4096^2 tuned fp32, t=99] e_rho={er:.3e} e_u={eu:.3e}", flush=True)
    assert er <= 1e-5 and eu <= 1e-5
