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
    mc = torch.empty((n, 4), device="cuda")
    mom = torch.empty((n, 3), device="cuda")
    res = torch.empty((n, 3), device="cuda")
    lbm.lbm_closure_features(g.ctx, sd.data_ptr(), n, feat.data_ptr(), mc.data_ptr())
    lbm.lbm_closure_moments(g.ctx, sd.data_ptr(), n, None, mom.data_ptr())
    lbm.lbm_closure_moments(g.ctx, sd.data_ptr(), n, mc.data_ptr(), res.data_ptr())
    feat, mc, mom, res = feat.cpu().numpy(), mc.cpu().numpy(), mom.cpu().numpy(), res.cpu().numpy()
    post = o.post_collision()
    # fp64 store: the inputs are computed in fp64 and returned as fp32 (relative rounding 6e-8);
    # fp32 store: non-equilibrium moments are differences of O(1e-2) fp32 populations (~1e-9 each),
    # and every input but 81, 85, 86 is divided by the strip amplitude A
    rtol, atol = (1e-6, 1e-12) if store == "f64" else (2e-5, 5e-8)
    worst = 0.0
    for r, (x, y, e) in enumerate(s):
        of, omc, amp = OC.site_features(o, x, y, e, gamma=0.6, beta=0.3, m0=(1.0005, 0.05, 0.02), post=post)
        err = np.abs(feat[r] - of) - rtol * np.abs(of)
        err[:85] *= amp  # back to unscaled units
        worst = max(worst, float(err.max()))
        assert np.all(err <= atol), (store, x, y, e, int(np.argmax(err)), float(err.max()))
        e_n = OC.NORMALS[e]
        refn = np.array([0.0005, 0.05 * e_n[0] + 0.02 * e_n[1], -0.05 * e_n[1] + 0.02 * e_n[0]])
        assert np.allclose(mc[r, :3], omc - refn, rtol=rtol, atol=atol)
        assert mc[r, 3] == pytest.approx(amp, rel=max(rtol, 1e-6), abs=atol)
        om = OC.site_moments(o, x, y, e)
        assert np.allclose(mom[r], om, rtol=rtol, atol=max(atol, 1e-9))
        # (moments - m_c) / A at the same time step, both differences taken against m0
        assert np.allclose(res[r] * amp, om - omc, rtol=1e-4, atol=2 * atol)
    print(f"\n[closure inputs {store}] worst excess over rtol: {worst:.2e}", flush=True)
    # a site whose strip leaves the lattice gives NaN
    bad = torch.tensor([[0, 0, 1, 0]], dtype=torch.int32, device="cuda")
    fb = torch.empty((1, 96), device="cuda")
    mb = torch.empty((1, 4), device="cuda")
    lbm.lbm_closure_features(g.ctx, bad.data_ptr(), 1, fb.data_ptr(), mb.data_ptr())
    assert torch.isnan(fb).all() and torch.isnan(mb).all()


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
    # element by element, per output against that output's largest magnitude
    err = (np.abs(y - yo) / np.abs(yo).max(axis=0)).max(axis=0)
    print(f"\n[mlp forward] max error per output / its max: {err}", flush=True)
    assert (err < 1e-3).all(), err


def test_gradients_match_oracle():
    """GPU gradients (BF16 MFMA, FP32 accumulation) against the fp64 oracle with the same BF16
    rounding points, element by element: every entry within 1e-3 of its tensor's largest entry.  FP32
    accumulation over 1000 samples and tanh differences that flip a BF16 activation rounding stay
    well below that; a wrong entry, a transposed block or a dropped term does not."""
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
        elem = np.abs(gu[k] - go[k]).max() / np.abs(go[k]).max()
        print(f"  grad {k}: norm rel err {rel:.2e}, max element err / max {elem:.2e}", flush=True)
        assert gu[k].shape == go[k].shape, k
        assert elem < 1e-3, (k, elem)


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


def test_closure_with_overlapped_edge_kernel_matches_serial():
    """The closure edge kernel on a second stream beside the bulk kernel gives the bits of the serial
    launches (a network with non-zero outputs, so the closure really acts)."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    blob = _trainer(_oracle_params(3)).export(6.0)
    nx, ny = 150, 70
    f = W.lamb_oseen(nx, ny, 60.0, 35.0, 6.0, 0.03, (0.05, 0.0))
    a = Lattice(nx, ny, 0.6, f, store="f32", m0=(1.0, 0.05, 0.0))
    b = Lattice(nx, ny, 0.6, f, store="f32", m0=(1.0, 0.05, 0.0))
    for g in (a, b):
        lbm.lbm_set_closure(g.ctx, blob.data_ptr(), 1)
    lbm.lbm_set_overlap(a.ctx, True)
    for n in (1, 6, 31):
        a.step(n)
        b.step(n)
        assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy()), n


def test_nonfinite_or_untrusted_output_falls_back_to_nsbc():
    p = _zero_params()
    p["b3"] = np.array([np.nan, 0.0, 0.0])
    a, b, _ = _closure_pair(p)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())
    a, b, _ = _closure_pair(_zero_params((7.0, 0.0, 0.0)), trust=6.0)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())


def test_constant_output_shifts_boundary_moments():
    """A network whose output is a constant c shifts every single-normal NSBC node's moments after one
    step by A c (normal frame, unit output scales; A the node's strip amplitude at time t); corners
    keep NSBC."""
    from paper_2005_08674_amd.lattice import Lattice
    from paper_2005_08674_amd import lbm
    c = (2e-2, 1e-1, -5e-2)
    tr = _trainer(_zero_params(c))
    blob = tr.export(6.0)
    nx, ny = 64, 48
    f = W.lamb_oseen(nx, ny, 30.0, 25.0, 5.0, 0.03, (0.05, 0.0))
    a = Lattice(nx, ny, 0.6, f, store="f64", m0=(1.0, 0.05, 0.0))
    b = Lattice(nx, ny, 0.6, f, store="f64", m0=(1.0, 0.05, 0.0))
    a.step(3)
    b.step(3)
    sites = np.array(_eligible_sites(nx, ny), np.int32)
    sd = torch.from_numpy(np.concatenate([sites, np.zeros((len(sites), 1), np.int32)], 1)).cuda()
    feat = torch.empty((len(sites), 96), device="cuda")
    mc = torch.empty((len(sites), 4), device="cuda")
    lbm.lbm_closure_features(b.ctx, sd.data_ptr(), len(sites), feat.data_ptr(), mc.data_ptr())
    amp = mc[:, 3].double().cpu().numpy()
    assert amp.min() > 0
    lbm.lbm_set_closure(b.ctx, blob.data_ptr(), 1)
    a.step(1)
    b.step(1)
    ma, mb = a.moments_np(), b.moments_np()
    for r, (x, y, e) in enumerate(sites):
        nxv, nyv = OC.NORMALS[e]
        s_r, s_n, s_t = (amp[r] * v for v in c)
        want = (s_r, s_n * nxv - s_t * nyv, s_n * nyv + s_t * nxv)
        for k in range(3):
            # the shift is formed in fp32: relative rounding ~1e-7 of A c
            assert mb[k][y, x] - ma[k][y, x] == pytest.approx(want[k], rel=1e-5, abs=1e-12), (x, y, e, k)
    # corners and the interior are untouched
    for m_a, m_b in zip(ma, mb):
        for (x, y) in ((0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)):
            assert m_a[y, x] == pytest.approx(m_b[y, x], abs=1e-15)
        assert np.abs(m_a[1:-1, 1:-1] - m_b[1:-1, 1:-1]).max() < 1e-15


def _eligible_sites(nx, ny):
    """Every single-normal boundary node (corners excluded) as (x, y, edge)."""
    s = [(0, y, 0) for y in range(1, ny - 1)] + [(nx - 1, y, 1) for y in range(1, ny - 1)]
    s += [(x, 0, 2) for x in range(1, nx - 1)] + [(x, ny - 1, 3) for x in range(1, nx - 1)]
    return s


def _normalization(feats):
    """Input mean and 1/std as lbm_mlp_fit_normalization defines them: inputs 87..95, constant
    inputs and strip-node inputs whose spread is below 1e-3 of the largest spread of the same
    moment over the nine strip nodes get (0, 0)."""
    mean, sd = feats.mean(0), feats.std(0)
    used = (np.arange(96) < 87) & (sd > 1e-30) & (sd > 1e-7 * np.abs(mean))
    top = sd[:81].reshape(9, 9).max(0)
    used[:81] &= sd[:81] > 1e-3 * np.tile(top, 9)
    mean = np.where(used, mean, 0.0).astype(np.float32)
    inv = np.where(used, 1.0 / np.where(used, sd, 1.0), 0.0).astype(np.float32)
    return mean, inv


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_fit_normalization_matches_numpy(store):
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    nx, ny = 70, 50
    f = W.lamb_oseen(nx, ny, 30.0, 22.0, 5.0, 0.04, (0.05, 0.02))
    g = Lattice(nx, ny, 0.6, f, store=store, m0=(1.0, 0.05, 0.02))
    g.step(15)
    s = np.array(_eligible_sites(nx, ny), np.int32)
    sd = torch.from_numpy(np.concatenate([s, np.zeros((len(s), 1), np.int32)], 1)).cuda()
    feat = torch.empty((len(s), 96), device="cuda")
    mc = torch.empty((len(s), 4), device="cuda")
    lbm.lbm_closure_features(g.ctx, sd.data_ptr(), len(s), feat.data_ptr(), mc.data_ptr())
    resid = torch.tensor(np.random.default_rng(3).standard_normal((len(s), 3)) * [1e-5, 1e-4, 2e-4],
                         dtype=torch.float32, device="cuda")
    tr = _trainer(_zero_params())
    tr.fit_normalization(feat, resid)
    mean, inv, scale = tr.normalization()
    fn = feat.cpu().numpy().astype(np.float64)
    want_mean, want_inv = _normalization(fn)
    # Q_ntt of the boundary row, which NSBC's non-equilibrium bounce-back cancels, holds fp64
    # rounding noise only (in fp32 storage the noise can reach the floor's 1e-3)
    dropped = [q for q in range(81) if want_inv[q] == 0.0]
    if store == "f64":
        assert 7 in dropped and 16 in dropped and 25 in dropped, dropped
    assert np.allclose(mean, want_mean, rtol=1e-5, atol=1e-12)
    assert np.array_equal(inv == 0, want_inv == 0)
    assert np.allclose(inv, want_inv, rtol=1e-4)
    rn = resid.cpu().numpy().astype(np.float64)
    assert np.allclose(scale, np.sqrt((rn ** 2).mean(0)), rtol=1e-5)


@pytest.mark.parametrize("ubase", [(0.0, 0.0), (0.05, 0.02)])
def test_closure_in_edge_kernel_matches_oracle(ubase):
    """One closure step inside the edge kernel against the oracle: inputs from the oracle at time t
    (fp64), normalised, passed through the oracle network with the GPU's BF16 rounding points, added
    to m_c in the edge frame; the node's moments after the step must equal that vector (NSBC's
    assignment plus correction reproduces m_c exactly).  Corners and the interior follow NSBC."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    nx, ny, tau, beta, m0 = 70, 50, 0.6, 0.3, (1.0004, 0.05, 0.02)
    f = W.lamb_oseen(nx, ny, 30.0, 22.0, 5.0, 0.04, (0.05, 0.02))
    g = Lattice(nx, ny, tau, f, store="f64", beta=beta, m0=m0, ubase=ubase)
    o = oracle.Lattice(nx, ny, tau, *f, beta=beta, m0=m0)
    g.step(12)
    o.step(12)
    post = o.post_collision()
    sites = _eligible_sites(nx, ny)
    rows = [OC.site_features(o, x, y, e, gamma=0.6, beta=beta, m0=m0, post=post) for x, y, e in sites]
    feats = np.array([r[0] for r in rows])
    mcs = np.array([r[1] for r in rows])
    amps = np.array([r[2] for r in rows])
    mean, inv = _normalization(feats)
    scale = np.array([0.1, 0.2, 0.2], np.float32)
    p = _oracle_params(21)
    tr = _trainer(p)
    tr.set_normalization(mean, inv, scale)
    blob = tr.export(1e4)
    # oracle side: the GPU forms (float(x) - mean) * inv_std in fp32 before rounding to BF16
    xn = (feats.astype(np.float32) - mean) * inv
    y, _ = M.forward(p, xn.astype(np.float64), bf16=True)
    corr = y * scale.astype(np.float64) * amps[:, None]
    lbm.lbm_set_closure(g.ctx, blob.data_ptr(), 1)
    g.step(1)
    o.step(1)
    mg = g.moments_np()
    mo = o.moments()
    worst = 0.0
    for r, (x, y_, e) in enumerate(sites):
        nxv, nyv = OC.NORMALS[e]
        dr, un, ut = mcs[r] + corr[r]
        want = (dr, un * nxv - ut * nyv, un * nyv + ut * nxv)
        got = (mg[0][y_, x], mg[1][y_, x], mg[2][y_, x])
        err = max(abs(a - b) / (amps[r] * s) for a, b, s in zip(got, want, (scale[0], scale[1], scale[1])))
        worst = max(worst, err)
        assert err < 5e-3, (x, y_, e, got, want)
    print(f"\n[closure in edge kernel] worst error / output scale: {worst:.2e}; "
          f"max |correction| / scale: {np.abs(y).max():.2f}", flush=True)
    assert np.abs(y).max() > 0.3  # the network's correction is not trivially small
    # corners keep NSBC; the interior does not see the boundary within one step
    for c in range(3):
        for (x, y_) in ((0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1)):
            assert mg[c][y_, x] == pytest.approx(mo[c][y_, x], abs=1e-13)
        assert np.abs(mg[c][1:-1, 1:-1] - mo[c][1:-1, 1:-1]).max() < 1e-13


def test_ensemble_closure_matches_standalone():
    """Members running the closure inside the batched ensemble (one member on NSBC, the others on the
    network) are bit-identical to the same lattices stepped alone, eagerly and through graphs."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.ensemble import Ensemble, member_params
    from paper_2005_08674_amd.lattice import Lattice
    p = _oracle_params(31)
    tr = _trainer(p)
    tr.set_normalization(np.zeros(96, np.float32), np.full(96, 0.5, np.float32), np.full(3, 0.05, np.float32))
    blob = tr.export(4.0)
    specs = [(90, 70, 0.6, (0.05, 0.01)), (130, 64, 0.55, (0.0, 0.0)), (64, 140, 0.7, (-0.03, 0.04))]
    members, fields, far = [], [], []
    for nx, ny, tau, u0 in specs:
        members.append(member_params(nx, ny, tau, store="f32", ubase=u0))
        fields.append(W.lamb_oseen(nx, ny, nx * 0.6, ny * 0.45, 6.0, 0.03, u0))
        far.append((0.0, 1.0, u0[0], u0[1]))
    ens = Ensemble(members, fields)
    for k, fa in enumerate(far):
        ens.set_farfield(k, *fa)
    lbm.lbm_ens_set_closure(ens.ens, -1, blob.data_ptr(), 1)
    lbm.lbm_ens_set_closure(ens.ens, 1, None, 0)
    ens.step(5)
    ens.step_graph(20)
    for k, (pm, f) in enumerate(zip(members, fields)):
        g = Lattice(pm.nx, pm.ny, pm.tau, f, store="f32", m0=far[k][1:], ubase=(pm.ubase[0], pm.ubase[1]))
        if k != 1:
            lbm.lbm_set_closure(g.ctx, blob.data_ptr(), 1)
        g.step(25)
        assert np.array_equal(ens.populations(k), g.populations().cpu().numpy()), k
        g.close()
    # the closure changed the members that run it
    h = Lattice(members[0].nx, members[0].ny, members[0].tau, fields[0], store="f32", m0=far[0][1:],
                ubase=(members[0].ubase[0], members[0].ubase[1]))
    h.step(25)
    assert not np.array_equal(ens.populations(0), h.populations().cpu().numpy())


def test_trained_closure_beats_nsbc_one_step_on_heldout_members():
    """Train on the ensemble members' NSBC edges with paired-twin targets (a small version of the
    48-member, 800-step workload) and check the one-step error on held-out members: the network's
    mean squared residual is below half of NSBC's."""
    from paper_2005_08674_amd.closure import Trainer, generate_dataset, heldout_mse
    members = W.ensemble_members(48, seed=4)
    held = W.ensemble_members(8, seed=40)
    f, r = generate_dataset(members, W.member_fields, W.member_m0, steps=800, log_every=10, stride=4, amp_rel=0.1)
    hf, hr = generate_dataset(held, W.member_fields, W.member_m0, steps=800, log_every=10, stride=4, amp_rel=0.1)
    assert f.shape[0] > 50000 and hf.shape[0] > 5000
    tr = Trainer(max_batch=4096)
    tr.fit_normalization(f, r)
    x, t = tr.pack(f, r)
    losses = tr.train(x, t, epochs=10, batch=4096, lr=2e-3, lr_end=1e-4)
    hx, ht = tr.pack(hf, hr)
    mse = heldout_mse(tr, hx, ht)
    mse0 = float((ht.double() ** 2).mean().item())
    print(f"\n[closure one-step, held-out] MSE network {mse:.4f} vs NSBC {mse0:.4f} "
          f"(gain {1 - mse / mse0:.3f}); train loss {losses[0]:.3f} -> {losses[-1]:.3f}", flush=True)
    assert mse < 0.5 * mse0


def test_regime_gate_selects_vortical_nodes():
    """With the regime gate kmin, a constant-output network shifts a boundary node's moments by A c only
    where the strip's kinetic disturbance exceeds kmin times its acoustic part (computed here from the
    oracle's inputs): nodes near a convected vortex are corrected, nodes reached by a sound pulse keep
    NSBC."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    nx, ny, u0 = 96, 80, (0.05, 0.0)
    fv = W.lamb_oseen(nx, ny, 10.0, 40.0, 5.0, 0.03, u0)
    fp = W.gaussian_pulses(nx, ny, [(1e-3, 4.0, 80.0, 40.0)])
    f = (fv[0] + fp[0], fv[1], fv[2])
    m0 = (1.0, u0[0], u0[1])
    c = (0.05, 0.1, -0.08)
    kmin = 10.0
    tr = _trainer(_zero_params(c))
    blob = tr.export(6.0, 1.0, kmin)
    a = Lattice(nx, ny, 0.6, f, store="f64", m0=m0, ubase=u0)
    b = Lattice(nx, ny, 0.6, f, store="f64", m0=m0, ubase=u0)
    o = oracle.Lattice(nx, ny, 0.6, *f, m0=m0)
    a.step(24)
    b.step(24)
    o.step(24)
    post = o.post_collision()
    lbm.lbm_set_closure(b.ctx, blob.data_ptr(), 1)
    a.step(1)
    b.step(1)
    ma, mb = a.moments_np(), b.moments_np()
    n_on = n_off = 0
    for (x, y, e) in _eligible_sites(nx, ny):
        feat, _, amp = OC.site_features(o, x, y, e, gamma=0.6, m0=m0, post=post)
        s = feat[:81].reshape(9, 9)
        k = (s[:, 1] ** 2 + s[:, 2] ** 2).sum() / ((s[:, 0] ** 2).sum() / 3.0)
        if abs(k / kmin - 1.0) < 0.02 or amp < 1e-9:
            continue  # borderline or no disturbance: either decision is valid
        nxv, nyv = OC.NORMALS[e]
        want = (amp * c[0], amp * (c[1] * nxv - c[2] * nyv), amp * (c[1] * nyv + c[2] * nxv))
        got = tuple(mb[q][y, x] - ma[q][y, x] for q in range(3))
        if k > kmin:
            n_on += 1
            assert np.allclose(got, want, rtol=1e-4, atol=1e-12), (x, y, e, k, got, want)
        else:
            n_off += 1
            assert max(abs(v) for v in got) == 0.0, (x, y, e, k, got)
    print(f"\n[regime gate kmin={kmin}] corrected {n_on} vortical nodes, left {n_off} acoustic nodes on NSBC",
          flush=True)
    assert n_on > 10 and n_off > 10


THREE_STEP_STORES = ["f64", "f32", "f16", "bf16"]


@pytest.mark.parametrize("store", THREE_STEP_STORES)
def test_closure_in_three_step_sweep_is_bit_identical(store):
    """The three-step sweep with the closure in its edge tiles gives the bits of closure single steps,
    for every three-step shape the lattice takes, on lattices one tile wide (both columns in a tile),
    ragged in both directions and with u_b != 0; a remainder of two steps runs as closure single
    steps.  The network (random weights, every single-normal edge node accepted) changes the result."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    p = _oracle_params(47)
    tr = _trainer(p)
    tr.set_normalization(np.zeros(96, np.float32), np.full(96, 0.5, np.float32), np.full(3, 0.02, np.float32))
    blob = tr.export(50.0, 1.0, 0.0)
    names = [lbm.lbm_two_step_describe(i) for i in range(lbm.lbm_two_step_count())]
    three = [i for i, n in enumerate(names) if n.startswith("3step")]
    cases = [(64, 40, (0.04, 0.01)), (131, 77, (0.0, 0.0)), (200, 150, (-0.03, 0.05))]
    for nx, ny, u0 in cases:
        # a vortex on the right edge and a pulse at the bottom-left corner: disturbed edges from t = 0
        dv, ux, uy = W.lamb_oseen(nx, ny, nx - 6.0, ny * 0.45, 5.0, 0.03, u0)
        dp, _, _ = W.gaussian_pulses(nx, ny, [(1e-3, 6.0, 5.0, 4.0)])
        f = (dv + dp, ux, uy)
        kw = dict(store=store, m0=(1.0, u0[0], u0[1]), ubase=u0, beta=0.1)
        ref = Lattice(nx, ny, 0.58, f, **kw)
        lbm.lbm_set_closure(ref.ctx, blob.data_ptr(), 1)
        ref.step(11)
        want = ref.populations().cpu().numpy()
        plain = Lattice(nx, ny, 0.58, f, **kw)
        plain.step(11)
        assert not np.array_equal(want, plain.populations().cpu().numpy())
        plain.close()
        ran = 0
        for sid in three:
            g = Lattice(nx, ny, 0.58, f, **kw)
            lbm.lbm_set_closure(g.ctx, blob.data_ptr(), 1)
            try:
                lbm.lbm_set_two_step(g.ctx, sid)
            except lbm.LbmError:
                g.close()
                continue
            lbm.lbm_enable_timing(g.ctx, True)
            g.step(11)
            ms, launches = lbm.lbm_two_step_times(g.ctx)
            got = g.populations().cpu().numpy()
            g.close()
            # every shape the lattice takes also fits the closure's LDS (the two levels, the edge
            # nodes' outputs, the staged biases and normalisation, the phases' scratch)
            assert launches == 3, (names[sid], launches)
            ran += 1
            assert np.array_equal(got, want), (nx, ny, names[sid])
        ref.close()
        assert ran > 0


@pytest.mark.parametrize("store", ["f32", "f16"])
def test_closure_launch_chain_is_bit_identical(store):
    """Ten closure launches in one lbm_step (the edge-tile kernel on the second stream joined only
    once, at the end) on a ragged square lattice whose inner strips border the edge tiles on all
    four sides give the bits of closure single steps, for a march shape and a tile shape; the
    same launches one lbm_step at a time agree too."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    p = _oracle_params(53)
    tr = _trainer(p)
    tr.set_normalization(np.zeros(96, np.float32), np.full(96, 0.5, np.float32), np.full(3, 0.02, np.float32))
    blob = tr.export(50.0, 1.0, 0.0)
    names = [lbm.lbm_two_step_describe(i) for i in range(lbm.lbm_two_step_count())]
    nx, ny, u0 = 520, 460, (0.05, -0.02)
    dv, ux, uy = W.lamb_oseen(nx, ny, nx - 8.0, ny * 0.4, 6.0, 0.03, u0)
    dp, _, _ = W.gaussian_pulses(nx, ny, [(1e-3, 6.0, 6.0, 5.0), (1e-3, 6.0, nx * 0.5, ny - 6.0)])
    f = (dv + dp, ux, uy)
    kw = dict(store=store, m0=(1.0, u0[0], u0[1]), ubase=u0, beta=0.1)
    ref = Lattice(nx, ny, 0.58, f, **kw)
    lbm.lbm_set_closure(ref.ctx, blob.data_ptr(), 1)
    ref.step(30)
    want = ref.populations().cpu().numpy()
    ref.close()
    shapes = ["3step:64x12/768+march11xh64+xcdband+nts", "3step:64x12/512+xcdband+nts", "3step:64x16/512+xcdband+nts"]
    ran = []
    for name in shapes:
        for per_call in (30, 3):
            g = Lattice(nx, ny, 0.58, f, **kw)
            lbm.lbm_set_closure(g.ctx, blob.data_ptr(), 1)
            try:
                lbm.lbm_set_two_step(g.ctx, names.index(name))
            except lbm.LbmError:  # a shape whose LDS cannot also hold the closure's
                g.close()
                continue
            for _ in range(30 // per_call):
                g.step(per_call)
            got = g.populations().cpu().numpy()
            g.close()
            ran.append(name)
            assert np.array_equal(got, want), (store, name, per_call)
    assert shapes[0] in ran


def test_closure_three_step_autotune_and_trained_network():
    """With the committed network: the two-step shapes are refused for closure lattices by the tuner
    (negative time), a three-step shape is chosen, and 2048 x 64 steps agree bit for bit with closure
    single steps."""
    import os
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.closure import Trainer
    from paper_2005_08674_amd.lattice import Lattice
    path = os.path.join(os.path.dirname(__file__), "..", "paper_2005_08674_amd", "data", "closure_c4.npz")
    blob = Trainer.load(path).export()
    nx, ny, u0 = 2048, 64, (0.1, 0.0)
    f = W.lamb_oseen(nx, ny, 2030.0, 30.0, 8.0, 0.02, u0)
    kw = dict(store="f32", m0=(1.0, 0.1, 0.0), ubase=u0)
    a = Lattice(nx, ny, 0.55, f, **kw)
    b = Lattice(nx, ny, 0.55, f, **kw)
    for g in (a, b):
        lbm.lbm_set_closure(g.ctx, blob.data_ptr(), 1)
    best, t = lbm.lbm_autotune_two_step(b.ctx, 2)
    names = [lbm.lbm_two_step_describe(i) for i in range(lbm.lbm_two_step_count())]
    assert names[best].startswith("3step")
    assert all(t[i] < 0 for i, n in enumerate(names) if n.startswith("2step"))
    a.step(30)
    b.step(30)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())
    a.close()
    b.close()
