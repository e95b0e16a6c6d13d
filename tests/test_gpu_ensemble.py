"""GPU ensemble: every member of a batched ensemble is bit-identical to the
same lattice stepped alone; graph replays equal eager steps; the 256-member
workload runs in one graph launch."""
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


def _mixed_members(store="f32"):
    """Uneven small lattices with every edge mix and reading variant."""
    from paper_2005_08674_amd.ensemble import member_params
    rng = np.random.default_rng(21)
    specs = [
        dict(nx=67, ny=45), dict(nx=130, ny=70, bc=(1, 1, 0, 0)), dict(nx=70, ny=130, bc=(0, 0, 1, 1)),
        dict(nx=65, ny=66, bc=(0, 0, 0, 0)), dict(nx=100, ny=90, grad_order=2), dict(nx=3, ny=3),
        dict(nx=3, ny=150, corner_mode=1), dict(nx=257, ny=64, corr_mode=1), dict(nx=64, ny=257),
        dict(nx=200, ny=3, bc=(1, 1, 0, 0)), dict(nx=333, ny=129, ubase=(0.05, -0.02)),
    ]
    members, fields, far = [], [], []
    for sp in specs:
        nx, ny = sp.pop("nx"), sp.pop("ny")
        tau = float(rng.uniform(0.52, 0.8))
        members.append(member_params(nx, ny, tau, store=store, **sp))
        u0 = (float(rng.uniform(-0.05, 0.05)), float(rng.uniform(-0.05, 0.05)))
        fields.append(W.gaussian_pulses(nx, ny, [(1e-3, 5.0, rng.uniform(0, nx), rng.uniform(0, ny))], u0=u0))
        far.append((float(rng.uniform(0, 0.5)), 1.0 + 1e-4, u0[0], u0[1]))
    return members, fields, far


def _standalone(p, f, far):
    from paper_2005_08674_amd.lattice import Lattice
    from paper_2005_08674_amd import lbm
    g = Lattice(p.nx, p.ny, p.tau, f, rho0=p.rho0, bc=tuple(p.bc), gamma=p.gamma, store=p.store,
                corr_mode=p.corr_mode, grad_order=p.grad_order, corner_mode=p.corner_mode,
                ubase=(p.ubase[0], p.ubase[1]))
    g.set_farfield(*far)
    return g


@pytest.mark.parametrize("store", ["f32", "f16", "f64"])
def test_members_bitwise_equal_standalone(store):
    from paper_2005_08674_amd.ensemble import Ensemble
    members, fields, far = _mixed_members(store)
    ens = Ensemble(members, fields)
    for m, fa in enumerate(far):
        ens.set_farfield(m, *fa)
    ens.step(13)
    for m, (p, f) in enumerate(zip(members, fields)):
        g = _standalone(p, f, far[m])
        g.step(13)
        assert np.array_equal(ens.populations(m), g.populations().cpu().numpy()), (store, m, p.nx, p.ny)
        g.close()


@pytest.mark.parametrize("store", ["f32", "f16", "f64"])
def test_fused_step_equals_separate_launches(store):
    """One launch per ensemble step gives the bits of separate bulk and edge launches, eagerly and
    through graphs, for every shape."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.ensemble import Ensemble
    members, fields, far = _mixed_members(store)
    for shape in range(lbm.lbm_ens_shape_count()):
        a = Ensemble(members, fields)
        b = Ensemble(members, fields)
        for m, fa in enumerate(far):
            a.set_farfield(m, *fa)
            b.set_farfield(m, *fa)
        lbm.lbm_ens_set_shape(a.ens, shape)
        lbm.lbm_ens_set_shape(b.ens, shape)
        lbm.lbm_ens_set_fused(b.ens, False)
        a.step(3)
        b.step(3)
        a.step_graph(4)
        b.step_graph(4)
        for m in range(len(members)):
            assert np.array_equal(a.populations(m), b.populations(m)), (store, shape, m)
        a.close()
        b.close()


def test_fp64_members_match_oracle():
    from paper_2005_08674_amd.ensemble import Ensemble
    members, fields, far = _mixed_members("f64")
    ens = Ensemble(members, fields)
    for m, fa in enumerate(far):
        ens.set_farfield(m, *fa)
    ens.step_graph(40)
    for m in (0, 4, 7, 10):
        p = members[m]
        o = oracle.Lattice(p.nx, p.ny, p.tau, *fields[m], bc=tuple(p.bc), gamma=p.gamma, beta=far[m][0],
                           m0=far[m][1:], corr_mode=p.corr_mode, grad_order=p.grad_order, corner_mode=p.corner_mode)
        o.step(40)
        gm, om = ens.moments(m), o.moments()
        assert np.abs(gm[0] - om[0]).max() < 1e-15
        assert max(np.abs(gm[1] - om[1]).max(), np.abs(gm[2] - om[2]).max()) / 0.05 < 1e-12


def test_graph_replays_equal_eager_steps():
    """Replay a captured 7-step graph repeatedly, with eager work and synchronisation between the
    replays and a far-field change, and check every replay against eager stepping."""
    from paper_2005_08674_amd.ensemble import Ensemble
    members, fields, far = _mixed_members("f32")
    a = Ensemble(members, fields)
    b = Ensemble(members, fields)
    for m, fa in enumerate(far):
        a.set_farfield(m, *fa)
        b.set_farfield(m, *fa)
    for rep in range(5):
        if rep == 3:
            a.set_farfield(2, 0.7, 1.0, 0.01, 0.0)
            b.set_farfield(2, 0.7, 1.0, 0.01, 0.0)
        a.step_graph(7)
        b.step(7)
        x = torch.randn(1000, device="cuda").sum().item()  # unrelated eager work between replays
        assert np.isfinite(x)
        for m in range(len(members)):
            assert np.array_equal(a.populations(m), b.populations(m)), (rep, m)
    assert a.t == b.t == 35


def test_all_shapes_bitwise_identical():
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.ensemble import Ensemble
    members, fields, far = _mixed_members("f32")
    ref = None
    for shape in range(lbm.lbm_ens_shape_count()):
        e = Ensemble(members, fields)
        lbm.lbm_ens_set_shape(e.ens, shape)
        e.step_graph(6)
        pops = [e.populations(m) for m in range(len(members))]
        if ref is None:
            ref = pops
        else:
            for m in range(len(members)):
                assert np.array_equal(pops[m], ref[m]), (shape, m)
        e.close()


def test_ensemble_256_one_graph_launch():
    """The 256-member workload (sizes U{64..512}^2, tau U[0.52, 0.8], pulse or vortex) in one graph
    launch of 200 steps; spot-check members against standalone lattices."""
    from paper_2005_08674_amd.ensemble import Ensemble, member_params
    ms = W.ensemble_members(256, seed=4)
    members = [member_params(m.nx, m.ny, m.tau, store="f32",
                             ubase=(m.params["u0"] if m.kind == "vortex" else (0.0, 0.0))) for m in ms]
    fields = [W.member_fields(m) for m in ms]
    ens = Ensemble(members, fields)
    for k, m in enumerate(ms):
        ens.set_farfield(k, 0.0, *W.member_m0(m))
    best, times = ens.autotune(reps=3)
    nodes, nb, ne = ens.info()
    ens.step_graph(200)  # capture + first launch
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ens.step_graph(200)
    e1.record()
    torch.cuda.synchronize()
    ms_ = e0.elapsed_time(e1)
    print(f"\n[ensemble 256] nodes={nodes} bulk blocks={nb} edge blocks={ne} shape={best} "
          f"{nodes * 200 / (ms_ * 1e-3) / 1e6:.0f} MLUPS ({ms_ / 200 * 1e3:.1f} us/step)", flush=True)
    for k in (0, 17, 255):
        g = _standalone(members[k], fields[k], (0.0, *W.member_m0(ms[k])))
        g.step(400)
        assert np.array_equal(ens.populations(k), g.populations().cpu().numpy()), k


def _nsbc_members(store, mrt_every=0):
    """Uneven lattices with NSBC on all four edges (what the two-step sweep needs), the reading
    variants, base velocity and, every `mrt_every`-th member, the MRT collision."""
    from paper_2005_08674_amd.ensemble import member_params
    rng = np.random.default_rng(41)
    specs = [dict(nx=67, ny=45), dict(nx=100, ny=90, grad_order=2), dict(nx=3, ny=3), dict(nx=3, ny=150, corner_mode=1),
             dict(nx=257, ny=64, corr_mode=1), dict(nx=64, ny=257), dict(nx=130, ny=3),
             dict(nx=333, ny=129, ubase=(0.05, -0.02)), dict(nx=65, ny=66)]
    members, fields, far = [], [], []
    for k, sp in enumerate(specs):
        nx, ny = sp.pop("nx"), sp.pop("ny")
        tau = float(rng.uniform(0.52, 0.8))
        mrt = (1.6, 1.4, 1.8) if mrt_every and k % mrt_every == 0 else None
        members.append(member_params(nx, ny, tau, store=store, mrt=mrt, **sp))
        u0 = (float(rng.uniform(-0.05, 0.05)), float(rng.uniform(-0.05, 0.05)))
        fields.append(W.gaussian_pulses(nx, ny, [(1e-3, 5.0, rng.uniform(0, nx), rng.uniform(0, ny))], u0=u0))
        far.append((float(rng.uniform(0, 0.5)), 1.0 + 1e-4, u0[0], u0[1]))
    return members, fields, far


@pytest.mark.parametrize("store", ["f32", "f16", "f64", "bf16"])
def test_two_step_equals_single_steps_every_shape(store):
    """The ensemble two-step sweep (one launch per two steps over every member's tiles) gives the bits of
    single steps for every shape, eagerly (with an odd step count) and through graphs."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.ensemble import Ensemble
    members, fields, far = _nsbc_members(store, mrt_every=3)
    ref = Ensemble(members, fields)
    for m, fa in enumerate(far):
        ref.set_farfield(m, *fa)
    ref.step(7)
    ref.step(8)
    want = [ref.populations(m) for m in range(len(members))]
    ref.close()
    for shape in range(lbm.lbm_two_step_count()):
        print(f"[ensemble multi-step] {store} {lbm.lbm_two_step_describe(shape)}", flush=True)
        e = Ensemble(members, fields)
        for m, fa in enumerate(far):
            e.set_farfield(m, *fa)
        if lbm.lbm_two_step_steps(shape) == 3 or "+march" in lbm.lbm_two_step_describe(shape):
            # these members include 3 x 3 and 130 x 3 lattices: three-step shapes are refused, and
            # the column marches take single lattices only
            with pytest.raises(lbm.LbmError):
                e.set_two_step(shape)
            e.close()
            continue
        e.set_two_step(shape)
        assert lbm.lbm_ens_get_two_step(e.ens) == shape
        e.step(7)
        e.step_graph(8)
        assert e.t == 15
        for m in range(len(members)):
            assert np.array_equal(e.populations(m), want[m]), (store, shape, m)
        e.close()


def test_two_step_graph_replays_and_autotune():
    """Replays of a captured two-step graph (odd length) with eager work and a far-field change between
    them match eager single steps; the autotuner leaves the state untouched and selects a shape."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.ensemble import Ensemble
    members, fields, far = _nsbc_members("f32")
    a = Ensemble(members, fields)
    b = Ensemble(members, fields)
    for m, fa in enumerate(far):
        a.set_farfield(m, *fa)
        b.set_farfield(m, *fa)
    best, times = a.autotune_two_step(reps=3)
    assert 0 <= best < lbm.lbm_two_step_count() == len(times)
    march = ["+march" in lbm.lbm_two_step_describe(k) for k in range(len(times))]
    assert min(t for k, t in enumerate(times) if lbm.lbm_two_step_steps(k) == 2 and not march[k]) > 0
    assert all(t < 0 for k, t in enumerate(times) if march[k])  # single lattices only
    assert a.t == 0
    for rep in range(4):
        if rep == 2:
            a.set_farfield(1, 0.7, 1.0, 0.01, 0.0)
            b.set_farfield(1, 0.7, 1.0, 0.01, 0.0)
        a.step_graph(9)
        b.step(9)
        x = torch.randn(1000, device="cuda").sum().item()
        assert np.isfinite(x)
        for m in range(len(members)):
            assert np.array_equal(a.populations(m), b.populations(m)), (rep, m)
    a.close()
    b.close()


def test_two_step_refused_with_periodic_member_and_off_with_closure():
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.ensemble import Ensemble
    members, fields, far = _mixed_members("f32")      # has periodic members
    e = Ensemble(members, fields)
    with pytest.raises(lbm.LbmError):
        e.set_two_step(0)
    with pytest.raises(lbm.LbmError):
        e.autotune_two_step(reps=1)
    e.set_two_step(-1)
    e.close()


@pytest.mark.parametrize("store", ["f32", "f64", "f16", "bf16"])
def test_three_step_ensemble_bitwise_equal_to_single_steps(store):
    """Members all at least 64 wide and 20 tall (the three-step sweep's condition), mixed BGK/MRT and
    reading variants: every three-step shape the format takes gives each member the bits of single
    steps, eagerly (11 steps: 3 launches + 2 single steps) and in a graph of 10 steps."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.ensemble import Ensemble, member_params
    rng = np.random.default_rng(43)
    specs = [dict(nx=67, ny=45), dict(nx=100, ny=90, grad_order=2), dict(nx=64, ny=20, corner_mode=1),
             dict(nx=257, ny=64, corr_mode=1), dict(nx=130, ny=33), dict(nx=65, ny=66, ubase=(0.04, -0.02))]
    members, fields, far = [], [], []
    for k, sp in enumerate(specs):
        nx, ny = sp.pop("nx"), sp.pop("ny")
        mrt = (1.6, 1.4, 1.8) if k % 2 else None
        members.append(member_params(nx, ny, float(rng.uniform(0.52, 0.8)), store=store, mrt=mrt, **sp))
        u0 = (float(rng.uniform(-0.05, 0.05)), float(rng.uniform(-0.05, 0.05)))
        fields.append(W.gaussian_pulses(nx, ny, [(1e-3, 5.0, rng.uniform(0, nx), rng.uniform(0, ny))], u0=u0))
        far.append((float(rng.uniform(0, 0.5)), 1.0 + 1e-4, u0[0], u0[1]))
    ref = Ensemble(members, fields)
    for m, fa in enumerate(far):
        ref.set_farfield(m, *fa)
    ref.step(11)
    want11 = [ref.populations(m) for m in range(len(members))]
    ref.step(10)
    want21 = [ref.populations(m) for m in range(len(members))]
    ref.close()
    for shape in range(lbm.lbm_two_step_count()):
        if lbm.lbm_two_step_steps(shape) != 3:
            continue
        ty = int(lbm.lbm_two_step_describe(shape).split("x")[1].split("/")[0])
        e = Ensemble(members, fields)
        for m, fa in enumerate(far):
            e.set_farfield(m, *fa)
        if (9 * ((ty + 4) * 68 + (ty + 2) * 66) * {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[store] > 160 * 1024
                or ty > 20 or "+march" in lbm.lbm_two_step_describe(shape)):
            # the two LDS levels do not fit, a member (64 x 20) is shorter than the tile, or the shape
            # is a column march (single lattices only)
            with pytest.raises(lbm.LbmError):
                e.set_two_step(shape)
            e.close()
            continue
        print(f"[ensemble three-step] {store} {lbm.lbm_two_step_describe(shape)}", flush=True)
        e.set_two_step(shape)
        e.step(11)
        for m in range(len(members)):
            assert np.array_equal(e.populations(m), want11[m]), (store, shape, m)
        e.step_graph(10)
        assert e.t == 21
        for m in range(len(members)):
            assert np.array_equal(e.populations(m), want21[m]), (store, shape, m)
        e.close()


def _member_and_twin_ensemble(members, steps_shape=True):
    """Members of `members` plus one twin each (padded N/2 per side, same analytic field), far field set
    as the closure data generation does; returns (Ensemble, member sites, twin sites)."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.closure import edge_sites, twin_fields
    from paper_2005_08674_amd.ensemble import Ensemble, member_params
    lat, fields, ms, ts = [], [], [], []
    for k, m in enumerate(members):
        u0 = W.member_m0(m)[1:]
        lat.append(member_params(m.nx, m.ny, m.tau, ubase=u0 if m.kind == "vortex" else (0.0, 0.0)))
        fields.append(W.member_fields(m))
        s = edge_sites(m.nx, m.ny, 3)
        ms.append(np.concatenate([np.full((len(s), 1), k, np.int32), s], 1))
    for k, m in enumerate(members):
        u0 = W.member_m0(m)[1:]
        px, py = m.nx // 2, m.ny // 2
        lat.append(member_params(m.nx + 2 * px, m.ny + 2 * py, m.tau,
                                 ubase=u0 if m.kind == "vortex" else (0.0, 0.0)))
        fields.append(twin_fields(W.member_fields, m, px, py))
        t = ms[k].copy()
        t[:, 0] = len(members) + k
        t[:, 1] += px
        t[:, 2] += py
        ts.append(t)
    ens = Ensemble(lat, fields)
    for k, m in enumerate(members):
        ens.set_farfield(k, 0.0, *W.member_m0(m))
        ens.set_farfield(len(members) + k, 0.0, *W.member_m0(m))
    if steps_shape:
        three = [i for i in range(lbm.lbm_two_step_count()) if lbm.lbm_two_step_describe(i).startswith("3step:64x12/768")]
        ens.set_two_step(three[0])
    cat = lambda a: torch.from_numpy(np.ascontiguousarray(np.concatenate(a))).to("cuda")
    return ens, cat(ms), cat(ts)


def test_graph_logging_equals_eager_sampling():
    """lbm_ens_step_graph with a log buffer writes, every log_every steps, exactly what the sampling
    calls (lbm_ens_closure_features / lbm_ens_closure_moments) return between eager steps: the closure
    inputs at time t, m_c and A, and the twin's residual target at t + 1.  The members end in the same
    state, and a replay of the cached graph from the new state matches eager sampling again."""
    from paper_2005_08674_amd import lbm
    members = W.ensemble_members(6, seed=11, lo=64, hi=120)
    a, ms, ts = _member_and_twin_ensemble(members)
    b, _, _ = _member_and_twin_ensemble(members)
    a.set_log_sites(ms, ts)
    n_sites = ms.shape[0]
    for rep in range(2):
        steps, every = 47, 10
        f, mc, r = a.step_graph_logged(steps, every)
        torch.cuda.synchronize()
        assert f.shape == (5, n_sites, 96) and mc.shape == (5, n_sites, 4) and r.shape == (5, n_sites, 3)
        for j in range(5):
            fe = torch.empty((n_sites, 96), dtype=torch.float32, device="cuda")
            me = torch.empty((n_sites, 4), dtype=torch.float32, device="cuda")
            re = torch.empty((n_sites, 3), dtype=torch.float32, device="cuda")
            lbm.lbm_ens_closure_features(b.ens, ms.data_ptr(), n_sites, fe.data_ptr(), me.data_ptr())
            b.step(1)
            lbm.lbm_ens_closure_moments(b.ens, ts.data_ptr(), n_sites, me.data_ptr(), re.data_ptr())
            b.step(min(every - 1, steps - every * j - 1))
            torch.cuda.synchronize()
            print(f"[graph log] replay {rep} record {j}", flush=True)
            # sites with no disturbance yet (A = 0) give NaN residuals on both sides: compare the bits
            assert torch.isfinite(fe).all() and torch.isfinite(re).any()
            bits = lambda x: x.contiguous().view(torch.int32)
            assert torch.equal(bits(f[j]), bits(fe)) and torch.equal(bits(mc[j]), bits(me)), (rep, j)
            assert torch.equal(bits(r[j]), bits(re)), (rep, j)
        assert a.t == b.t == steps * (rep + 1)
        for k in range(2 * len(members)):
            assert np.array_equal(a.populations(k), b.populations(k)), (rep, k)
    # refusals: a buffer that is too small, and logging without sites
    nbytes = lbm.lbm_ens_log_bytes(a.ens, 47, 10)
    assert nbytes == 5 * n_sites * 103 * 4
    small = torch.empty(nbytes // 4 - 1, dtype=torch.float32, device="cuda")
    with pytest.raises(lbm.LbmError):
        lbm.lbm_ens_step_graph(a.ens, 47, small.data_ptr(), small.numel() * 4, 10)
    lbm.lbm_ens_set_log_sites(a.ens, None, None, 0)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_ens_step_graph(a.ens, 47, small.data_ptr(), nbytes, 10)
    assert e.value.code == lbm.LBM_ERR_STATE
    a.close()
    b.close()
