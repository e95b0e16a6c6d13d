"""GPU reflection measurement: the fp64 energy reduction against numpy, the
reflection coefficient of the 128^2 pulse against the oracle's, the gamma
sweep, the storage precisions, and the convected vortex."""
import math

import numpy as np
import pytest

import oracle
from oracle import reflection as OR
from paper_2005_08674_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_08674_amd import lbm
    lbm.load()


def _pulse_fn(a=1e-3, w=6.0, xc=63.5, yc=63.5, u0=(0.0, 0.0)):
    def fn(x, y):
        d = a * np.exp(-math.log(2.0) * ((x - xc) ** 2 + (y - yc) ** 2) / (w * w))
        return d, np.full_like(x, u0[0]), np.full_like(x, u0[1])
    return fn


def test_energy_reduction_matches_numpy():
    from paper_2005_08674_amd.lattice import Lattice
    rng = np.random.default_rng(11)
    nx, ny, NX, NY, ox, oy = 77, 53, 200, 150, 31, 47
    f = (1e-3 * rng.standard_normal((ny, nx)), 0.01 * rng.standard_normal((ny, nx)),
         0.01 * rng.standard_normal((ny, nx)))
    F = (1e-3 * rng.standard_normal((NY, NX)), 0.01 * rng.standard_normal((NY, NX)),
         0.01 * rng.standard_normal((NY, NX)))
    for store in ("f64", "f32", "f16"):
        t = Lattice(nx, ny, 0.6, f, store=store)
        r = Lattice(NX, NY, 0.6, F, store=store)
        t.step(3)
        r.step(3)
        mt, mr = t.moments_np(), r.moments_np()
        got = float(t.energy(r, ox, oy).item())
        want = OR.energy_diff(mt, OR.window(mr, ox, oy, nx, ny))
        assert got == pytest.approx(want, rel=1e-12), store
        got0 = float(t.energy(ux_ref=0.02, uy_ref=-0.01).item())
        want0 = OR.energy(mt[0], mt[1] - 0.02, mt[2] + 0.01)
        assert got0 == pytest.approx(want0, rel=1e-12), store


def _oracle_series(gamma, every=5, n=128):
    m = 4 * n
    off = (m - n) // 2
    fn = _pulse_fn(xc=(n - 1) / 2, yc=(n - 1) / 2)
    from paper_2005_08674_amd.reflection import fields_on, clean_time
    ft, fr = fields_on(fn, n, n), fields_on(fn, m, m, -off, -off)
    T = int(clean_time(m, m, n, n))
    e0 = OR.energy(*ft)
    t = oracle.Lattice(n, n, 0.6, *ft, gamma=gamma)
    r = oracle.Lattice(m, m, 0.6, *fr, gamma=gamma)
    out = []
    for k in range(T // every + 1):
        out.append(OR.energy_diff(t.moments(), OR.window(r.moments(), off, off, n, n)) / e0)
        if k < T // every:
            t.step(every)
            r.step(every)
    return np.array(out)


def test_pulse128_reflection_matches_oracle():
    """128^2 fp64, tau 0.6, gamma 0.6 vs a 512^2 reference: the GPU's R_E series equals the oracle's."""
    from paper_2005_08674_amd.reflection import ReflectionRun
    run = ReflectionRun(_pulse_fn(), 128, 128, 0.6, store="f64")
    res = run.run(2000, every=5)
    ors = _oracle_series(0.6)
    print(f"\n[reflection 128^2 fp64] R_E gpu={res['R_E']:.6e} oracle={ors.max():.6e} horizon={res['horizon']}",
          flush=True)
    assert len(ors) == len(res["series"])
    assert np.abs(res["series"] - ors).max() < 1e-10
    assert res["R_E"] < 1e-3


def test_gamma_sweep_on_gpu():
    """The best gamma of the paper (0.6 for D2Q9) minimises the measured reflection."""
    from paper_2005_08674_amd.reflection import ReflectionRun
    r = {}
    for g in (0.4, 0.5, 0.6, 0.7, 0.8):
        run = ReflectionRun(_pulse_fn(), 128, 128, 0.6, store="f32", test_kw=dict(gamma=g),
                            ref_kw=dict(gamma=0.6))
        r[g] = run.run(2000, every=5)["R_E"]
        run.close()
    print("\n[gamma sweep fp32] " + " ".join(f"{g}:{v:.3e}" for g, v in r.items()), flush=True)
    assert min(r, key=r.get) == 0.6
    assert r[0.6] < 1e-3


@pytest.mark.parametrize("store,bar", [("f32", 1e-3), ("f16", 1e-3), ("bf16", 3e-3)])
def test_pulse128_reflection_by_storage(store, bar):
    """R_E of the 128^2 pulse with the test lattice stored in fp32/fp16/bf16 deviations against
    an fp64 reference: storage rounding adds to the measured reflection; reported per run."""
    from paper_2005_08674_amd.reflection import ReflectionRun
    run = ReflectionRun(_pulse_fn(), 128, 128, 0.6, store=store, ref_store="f64")
    res = run.run(2000, every=5)
    f64 = ReflectionRun(_pulse_fn(), 128, 128, 0.6, store="f64").run(2000, every=5)
    print(f"\n[reflection 128^2 {store}] R_E={res['R_E']:.4e} (fp64 {f64['R_E']:.4e})", flush=True)
    assert res["R_E"] < bar


def test_vortex512x256_is_absorbed():
    """512x256 fp32 vortex convected out through the right edge over 5000 steps, measured
    against a 2048x1024 reference: the energy of the difference stays a small fraction of the
    vortex's energy (the paper's "fully absorbed").  Bars a quarter above the measured values
    (R_E 1.61e-2, final 7.9e-5), so that a change to NSBC that reflects more fails here."""
    from paper_2005_08674_amd.reflection import ReflectionRun
    w = W.vortex_512x256()
    ex = w.extra

    def fn(x, y):
        return W.lamb_oseen_xy(x, y, ex["x0"], ex["y0"], ex["rc"], ex["uv"], (0.1, 0.0))

    run = ReflectionRun(fn, 512, 256, 0.55, store="f32", u0=(0.1, 0.0), ubase=(0.1, 0.0))
    res = run.run(5000, every=50, respect_clean_time=False)
    s = res["series"]
    print(f"\n[vortex 512x256 fp32] R_E={res['R_E']:.4e} final={s[-1]:.4e} at t={res['horizon']}", flush=True)
    assert s[-1] < 1e-4
    assert res["R_E"] < 2e-2


def test_committed_closure_closed_loop_against_nsbc():
    """The committed closure network (trained on the 256-member ensemble, run with its saved trust
    bound, gain and regime gate) in closed loop against plain NSBC, each test lattice against its 4x
    reference.  Sound waves stay below the gate, so the two acoustic cases reflect as with NSBC (to
    1e-3); on the convected vortex the closure reflects at most half as much as NSBC (0.24x measured)."""
    import os
    from paper_2005_08674_amd.closure import Trainer
    from paper_2005_08674_amd.reflection import ReflectionRun
    path = os.path.join(os.path.dirname(__file__), "..", "paper_2005_08674_amd", "data", "closure_c4.npz")
    tr = Trainer.load(path)
    blob = tr.export()
    w = W.vortex_512x256()
    ex = w.extra

    def vfn(x, y):
        return W.lamb_oseen_xy(x, y, ex["x0"], ex["y0"], ex["rc"], ex["uv"], (0.1, 0.0))

    cases = {
        "pulse128": (dict(field_fn=_pulse_fn(), nx=128, ny=128, tau=0.6, store="f32"), 2000, 5, True),
        "pulse_on_flow": (dict(field_fn=_pulse_fn(5e-4, 8.0, 90.0, 60.0, (0.06, -0.03)), nx=200, ny=150, tau=0.56,
                               store="f32", u0=(0.06, -0.03), ubase=(0.06, -0.03)), 3000, 5, True),
        "vortex512x256": (dict(field_fn=vfn, nx=512, ny=256, tau=0.55, store="f32", u0=(0.1, 0.0),
                               ubase=(0.1, 0.0)), 5000, 50, False),
    }
    out = {}
    for name, (kw, steps, every, rc) in cases.items():
        a = ReflectionRun(**kw)
        ra = a.run(steps, every=every, respect_clean_time=rc)
        a.close()
        b = ReflectionRun(**kw, closure=blob)
        rb = b.run(steps, every=every, respect_clean_time=rc)
        finite = b.test.check_finite()
        b.close()
        out[name] = (ra["R_E"], rb["R_E"])
        print(f"\n[closure closed loop] {name}: R_E NSBC {ra['R_E']:.4e}, closure {rb['R_E']:.4e} "
              f"(ratio {rb['R_E'] / ra['R_E']:.3f})", flush=True)
        assert finite and np.isfinite(rb["R_E"]) and rb["R_E"] < 0.1
    for name in ("pulse128", "pulse_on_flow"):
        # equal up to the few rounding-noise nodes (A ~ 1e-12) whose tiny disturbance the gate may pass
        assert out[name][1] <= out[name][0] * (1.0 + 1e-3), name
    assert out["vortex512x256"][1] <= 0.5 * out["vortex512x256"][0]
