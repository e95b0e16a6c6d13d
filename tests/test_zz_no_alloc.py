"""The allocation-free energy reduction (lbm_energy_noalloc) against lbm_energy, through the C ABI:
the same fp64 value bit for bit (same kernels, same order of summation), on two calls in a row, the
second on a smaller input, with and without a reference lattice."""
import pytest

from paper_2005_08674_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_08674_amd import lbm
    lbm.load()


def _pair(test, ref, x_off, y_off, u_ref):
    from paper_2005_08674_amd import lbm
    a = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    b = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    rc = ref.ctx if ref is not None else None
    lbm.lbm_energy(test.ctx, rc, x_off, y_off, u_ref[0], u_ref[1], a.data_ptr())
    lbm.lbm_energy_noalloc(test.ctx, rc, x_off, y_off, u_ref[0], u_ref[1], b.data_ptr())
    torch.cuda.synchronize()
    return float(a.item()), float(b.item())


def test_noalloc_energy_equals_workspace_energy_on_two_calls():
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    # first call: a 300x200 window inside a 700x500 reference, both stepped 60 steps, the pulse close
    # enough to the window's left edge that the two differ by the edge's reflection
    big = W.gaussian_pulses(700, 500, [(1e-3, 8.0, 235.0, 255.0)], u0=(0.02, 0.0))
    win = tuple(f[150:350, 200:500] for f in big)
    ref = Lattice(700, 500, 0.6, big, store="f32")
    test = Lattice(300, 200, 0.6, win, store="f32")
    ref.step(60)
    test.step(60)
    a, b = _pair(test, ref, 200, 150, (0.0, 0.0))
    print(f"\n[noalloc] 300x200 window: {a!r} {b!r}", flush=True)
    assert a > 1e-12 and a == b
    a, b = _pair(test, None, 0, 0, (0.02, 0.0))
    assert a > 0 and a == b
    # second call, smaller input: a 40x30 FP64 lattice against the uniform state
    small = W.gaussian_pulses(40, 30, [(5e-4, 3.0, 20.0, 14.0)], u0=(0.01, -0.01))
    t2 = Lattice(40, 30, 0.7, small, store="f64")
    t2.step(5)
    a2, b2 = _pair(t2, None, 0, 0, (0.01, -0.01))
    print(f"[noalloc] 40x30: {a2!r} {b2!r}", flush=True)
    assert a2 > 0 and a2 == b2 and a2 != a
    # a window that does not fit is refused before anything is enqueued
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(lbm.LbmError):
        lbm.lbm_energy_noalloc(ref.ctx, test.ctx, 0, 0, 0.0, 0.0, out.data_ptr())
    for g in (ref, test, t2):
        g.close()
