"""GPU learned closure: sampled inputs against the oracle, the BF16 MFMA
network (forward, gradients, Adam) against the numpy oracle, training, and
the closure inside the edge kernel (zero network = NSBC, NSBC fallback, exact
output shift)."""
import math

import numpy as np
import pytest

import oracle
from oracle import closure as OC
from oracle import mlp as M
from paper_2005_08674_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2005_08674_amd import lbm
    lbm.load()


def _sites(nx, ny):
    from paper_2005_08674_amd.closure import edge_sites
    s = edge_sites(nx, ny, stride=3)
    inner = np.array([[10, 12, 0], [15, 9, 1], [20, 7, 2], [8, 20, 3]], np.int32)
    return np.concatenate([s, inner])


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_sampled_inputs_match_oracle(store):
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    nx, ny = 40, 32
    f = W.lamb_oseen(nx, ny, 17.0, 15.0, 5.0, 0.04, (0.05, 0.02))
    g = Lattice(nx, ny, 0.62, f, store=store, beta=0.3, m0=(1.0005, 0.05, 0.02))
    o = oracle.Lattice(nx, ny, 0.62, *f, beta=0.3, m0=(1.0005, 0.05, 0.02))
    g.step(9)
    o.step(9)
    s = _sites(nx, ny)
    sd = torch.from_numpy(np.concatenate([s, np.zeros((len(s), 1), np.int32)], 1)).cuda()
    n = len(s)
    feat = torch.empty((n, 96), device="cuda")
    mc = torch.empty((n, 3), device="cuda")
    mom = torch.empty((n, 3), device="cuda")
    lbm.lbm_closure_features(g.ctx, sd.data_ptr(), n, feat.data_ptr(), mc.data_ptr())
    lbm.lbm_closure_moments(g.ctx, sd.data_ptr(), n, None, mom.data_ptr())
    feat, mc, mom = feat.cpu().numpy(), mc.cpu().numpy(), mom.cpu().numpy()
    post = o.post_collision()
    # fp64 store: the inputs are computed in fp64 and returned as fp32 (relative rounding 6e-8);
    # fp32 store: non-equilibrium moments are differences of O(1e-2) fp32 populations (~1e-9 each)
    rtol, atol = (1e-6, 1e-12) if store == "f64" else (2e-5, 5e-8)
    worst = 0.0
    for r, (x, y, e) in enumerate(s):
        of, omc = OC.site_features(o, x, y, e, gamma=0.6, beta=0.3, m0=(1.0005, 0.05, 0.02), post=post)
        err = np.abs(feat[r] - of) - rtol * np.abs(of)
        worst = max(worst, float(err.max()))
        assert np.all(err <= atol), (store, x, y, e, int(np.argmax(err)), float(err.max()))
        assert np.allclose(mc[r], omc, rtol=rtol, atol=max(atol, 1e-9))
        assert np.allclose(mom[r], OC.site_moments(o, x, y, e), rtol=rtol, atol=max(atol, 1e-9))
    print(f"\n[closure inputs {store}] worst excess over rtol: {worst:.2e}", flush=True)
    # a site whose strip leaves the lattice gives NaN
    bad = torch.tensor([[0, 0, 1, 0]], dtype=torch.int32, device="cuda")
    fb = torch.empty((1, 96), device="cuda")
    mb = torch.empty((1, 3), device="cuda")
    lbm.lbm_closure_features(g.ctx, bad.data_ptr(), 1, fb.data_ptr(), mb.data_ptr())
    assert torch.isnan(fb).all()


def _bf16_inputs(n, seed):
    x = np.random.default_rng(seed).standard_normal((n, 96))
    x[:, 85:] = 0.0
    return M.bf16_round(x)


def _trainer(params, max_batch=1024):
    from paper_2005_08674_amd.closure import Trainer, pack_params
    return Trainer(pack_params(params), max_batch=max_batch)


def _oracle_params(seed):
    p = M.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    p["b1"] = 0.1 * rng.standard_normal(64)
    p["b2"] = 0.1 * rng.standard_normal(64)
    p["b3"] = 0.1 * rng.standard_normal(3)
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def test_forward_matches_oracle():
    p = _oracle_params(1)
    tr = _trainer(p)
    X = _bf16_inputs(333, 2)
    y = tr.forward(torch.tensor(X, dtype=torch.bfloat16, device="cuda")).cpu().numpy()
    yo, _ = M.forward(p, X, bf16=True)
    err = np.abs(y - yo).max() / np.abs(yo).max()
    print(f"\n[mlp forward] max rel err {err:.2e}", flush=True)
    assert err < 1e-2


def test_gradients_match_oracle():
    """Per-tensor relative error of the GPU gradients (BF16 MFMA, FP32 accumulation) against the
    fp64 oracle with the same BF16 rounding points."""
    from paper_2005_08674_amd.closure import unpack_params
    p = _oracle_params(3)
    tr = _trainer(p)
    X = _bf16_inputs(1000, 4)
    T = np.random.default_rng(5).standard_normal((1000, 3))
    g, loss = tr.grads(torch.tensor(X, dtype=torch.bfloat16, device="cuda"),
                       torch.tensor(T, dtype=torch.float32, device="cuda"))
    lo, go = M.loss_and_grads(p, X, T, bf16=True)
    assert loss == pytest.approx(lo, rel=1e-4)
    gu = unpack_params(g)
    for k in go:
        rel = np.linalg.norm(gu[k] - go[k]) / np.linalg.norm(go[k])
        print(f"  grad {k}: rel err {rel:.2e}", flush=True)
        assert rel < 2e-2, k


def test_adam_step_and_row_selection():
    """One Adam step equals the oracle's Adam applied to the GPU gradients; a row-index list
    selects exactly those samples."""
    from paper_2005_08674_amd.closure import pack_params, unpack_params
    p = _oracle_params(6)
    X = _bf16_inputs(512, 7)
    T = np.random.default_rng(8).standard_normal((512, 3))
    xd = torch.tensor(X, dtype=torch.bfloat16, device="cuda")
    td = torch.tensor(T, dtype=torch.float32, device="cuda")
    rows = torch.arange(255, -1, -1, dtype=torch.int32, device="cuda") * 2  # every other row, reversed
    a = _trainer(p)
    g_sel, _ = a.grads(xd, td, rows=rows)
    sub = _trainer(p)
    g_dir, _ = sub.grads(torch.tensor(X[::2][::-1].copy(), dtype=torch.bfloat16, device="cuda"),
                         torch.tensor(T[::2][::-1].copy(), dtype=torch.float32, device="cuda"))
    assert np.allclose(g_sel, g_dir, rtol=1e-5, atol=1e-9)
    a.train_step(xd, td, 1e-3, rows=rows)
    after = a.params()
    m0, v0 = M.adam_init(p)
    want, _, _ = M.adam_step({k: v for k, v in p.items()}, unpack_params(g_sel), m0, v0, 1, 1e-3)
    assert np.allclose(after, pack_params(want), rtol=1e-5, atol=1e-7)


def test_training_reduces_loss():
    """Fit a random teacher network: the loss falls by 5x or more in 300 Adam steps."""
    teacher = _oracle_params(9)
    X = _bf16_inputs(4096, 10)
    T, _ = M.forward(teacher, X, bf16=False)
    tr = _trainer(_oracle_params(11), max_batch=1024)
    xd = torch.tensor(X, dtype=torch.bfloat16, device="cuda")
    td = torch.tensor(T, dtype=torch.float32, device="cuda")
    losses = tr.train(xd, td, epochs=75, batch=1024, lr=3e-3, lr_end=3e-4)
    print(f"\n[mlp training] loss {losses[0]:.4f} -> {losses[-1]:.5f}", flush=True)
    assert losses[-1] < losses[0] / 5


def _closure_pair(net_params, trust=6.0, steps=25, store="f32"):
    """(NSBC lattice, closure lattice) stepped `steps` times from the same vortex field."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    tr = _trainer(net_params)
    blob = tr.export(trust)
    nx, ny = 150, 70
    f = W.lamb_oseen(nx, ny, 60.0, 35.0, 6.0, 0.03, (0.05, 0.0))
    a = Lattice(nx, ny, 0.6, f, store=store, m0=(1.0, 0.05, 0.0))
    b = Lattice(nx, ny, 0.6, f, store=store, m0=(1.0, 0.05, 0.0))
    lbm.lbm_set_closure(b.ctx, blob.data_ptr(), 1)
    a.step(steps)
    b.step(steps)
    return a, b, blob


def _zero_params(b3=(0.0, 0.0, 0.0)):
    p = {"W1": np.zeros((64, 96)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
         "W3": np.zeros((3, 64)), "b3": np.array(b3, dtype=np.float64)}
    return p


def test_zero_network_equals_nsbc():
    a, b, _ = _closure_pair(_zero_params())
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())


def test_nonfinite_or_untrusted_output_falls_back_to_nsbc():
    p = _zero_params()
    p["b3"] = np.array([np.nan, 0.0, 0.0])
    a, b, _ = _closure_pair(p)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())
    a, b, _ = _closure_pair(_zero_params((7.0, 0.0, 0.0)), trust=6.0)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())


def test_constant_output_shifts_boundary_moments():
    """A network whose output is a constant c shifts every single-normal NSBC node's moments after one
    step by c (normal frame, unit scales); corners keep NSBC."""
    from paper_2005_08674_amd.lattice import Lattice
    from paper_2005_08674_amd import lbm
    c = (2e-4, 1e-3, -5e-4)
    tr = _trainer(_zero_params(c))
    blob = tr.export(6.0)
    nx, ny = 64, 48
    f = W.lamb_oseen(nx, ny, 30.0, 25.0, 5.0, 0.03, (0.05, 0.0))
    a = Lattice(nx, ny, 0.6, f, store="f64", m0=(1.0, 0.05, 0.0))
    b = Lattice(nx, ny, 0.6, f, store="f64", m0=(1.0, 0.05, 0.0))
    lbm.lbm_set_closure(b.ctx, blob.data_ptr(), 1)
    a.step(1)
    b.step(1)
    ma, mb = a.moments_np(), b.moments_np()
    # left edge (normal (-1, 0), tangent (0, -1)): drho += c0, u_x -= c1, u_y -= c2
    assert np.allclose(mb[0][1:-1, 0] - ma[0][1:-1, 0], c[0], atol=1e-7)
    assert np.allclose(mb[1][1:-1, 0] - ma[1][1:-1, 0], -c[1], atol=1e-7)
    assert np.allclose(mb[2][1:-1, 0] - ma[2][1:-1, 0], -c[2], atol=1e-7)
    # top edge (normal (0, 1), tangent (-1, 0)): u_y += c1, u_x -= c2
    assert np.allclose(mb[2][-1, 1:-1] - ma[2][-1, 1:-1], c[1], atol=1e-7)
    assert np.allclose(mb[1][-1, 1:-1] - ma[1][-1, 1:-1], -c[2], atol=1e-7)
    # corners and the interior are untouched
    for m_a, m_b in zip(ma, mb):
        assert m_a[0, 0] == pytest.approx(m_b[0, 0], abs=1e-15)
        assert np.abs(m_a[1:-1, 1:-1] - m_b[1:-1, 1:-1]).max() < 1e-15
