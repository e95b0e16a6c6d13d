"""GPU parity: the HIP path (through the C ABI) against the CPU fp64 oracle on
the same seeded inputs.

Tolerances: fp64 storage 1e-12 and fp32 storage 1e-5, both relative --
e_rho = max|rho - rho_oracle| / rho0 and e_u = max|u - u_oracle| / U_ref with
U_ref the workload's velocity scale (max(|u0|, c_s A) for pulses)."""
import math

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


def _lattice(**kw):
    from paper_2005_08674_amd.lattice import Lattice
    return Lattice(**kw)


def _errors(gpu_m, orc_m, rho0, u_ref):
    er = np.abs(gpu_m[0] - orc_m[0]).max() / rho0
    eu = max(np.abs(gpu_m[1] - orc_m[1]).max(), np.abs(gpu_m[2] - orc_m[2]).max()) / u_ref
    return er, eu


def _run_pair(nx, ny, tau, fields, checkpoints, store, tol, u_ref, bc=(1, 1, 1, 1), gamma=0.6, beta=0.0,
              m0=(1.0, 0.0, 0.0), ubase=(0.0, 0.0), **kw):
    print(f"\n[parity] {nx}x{ny} store={store} bc={bc} gamma={gamma} beta={beta} ubase={ubase} {kw}", flush=True)
    g = _lattice(nx=nx, ny=ny, tau=tau, fields=fields, bc=bc, gamma=gamma, store=store, beta=beta, m0=m0,
                 ubase=ubase, **kw)
    o = oracle.Lattice(nx, ny, tau, *fields, bc=bc, gamma=gamma, beta=beta, m0=m0, **kw)
    worst = (0.0, 0.0)
    for t in checkpoints:
        g.step(t - g.t)
        o.step(t - o.t)
        er, eu = _errors(g.moments_np(), o.moments(), 1.0, u_ref)
        print(f"  t={t:5d} e_rho={er:.3e} e_u={eu:.3e}", flush=True)
        assert er <= tol and eu <= tol, (t, er, eu)
        worst = (max(worst[0], er), max(worst[1], eu))
    return worst


def test_pulse128_fp64_1000_steps():
    """128x128 fp64, tau 0.6, NSBC on all edges, centred pulse: within 1e-12 of the oracle up to t = 1000."""
    w = W.pulse_128()
    _run_pair(w.nx, w.ny, w.tau, w.fields, [1, 10, 100, 250, 500, 1000], "f64", 1e-12, w.u_ref)


UB = dict(ubase=(0.03, -0.02))


@pytest.mark.parametrize("nx,ny,bc,kw", [
    (67, 45, (1, 1, 1, 1), {}),
    (67, 45, (1, 1, 1, 1), UB),
    (130, 70, (1, 1, 0, 0), {}),
    (70, 130, (0, 0, 1, 1), UB),
    (65, 66, (0, 0, 0, 0), {}),
    (67, 45, (1, 1, 1, 1), dict(grad_order=2)),
    (67, 45, (1, 1, 1, 1), dict(corner_mode=1, **UB)),
    (67, 45, (1, 1, 1, 1), dict(corr_mode=1)),
    (67, 45, (1, 1, 1, 1), dict(corr_mode=1, **UB)),
    (3, 3, (1, 1, 1, 1), {}),
    (3, 200, (1, 1, 1, 1), dict(grad_order=2)),
    (200, 3, (1, 1, 0, 0), UB),
])
def test_fp64_variants(nx, ny, bc, kw):
    """Ragged tiles, periodic pairs, the alternative readings and the smallest lattices, fp64."""
    rng = np.random.default_rng(nx * 1000 + ny)
    pulses = [(1e-3, 5.0, rng.uniform(0, nx), rng.uniform(0, ny))]
    f = W.gaussian_pulses(nx, ny, pulses, u0=(0.03, -0.02))
    _run_pair(nx, ny, 0.58, f, [1, 7, 60, 200], "f64", 1e-12, 0.03, bc=bc, beta=0.3, m0=(1.0005, 0.03, -0.02), **kw)


def test_vortex512x256_fp32_1000_steps():
    """512x256 fp32, tau 0.55, inflow 0.1, Lamb-Oseen vortex, deviations stored about the inflow
    equilibrium: within 1e-5 of the oracle at every checkpoint up to t = 1000."""
    w = W.vortex_512x256()
    _run_pair(w.nx, w.ny, w.tau, w.fields, [1, 10, 100, 250, 500, 1000], "f32", 1e-5, w.u_ref, m0=w.m0,
              ubase=(0.1, 0.0))


@pytest.mark.parametrize("store,tol", [("f16", 2e-3), ("bf16", 2e-2)])
def test_vortex_sixteen_bit_with_base_flow(store, tol):
    """256x128 vortex on an inflow of 0.1 stored about the inflow equilibrium in FP16 and BF16:
    interior nodes take the stored-form collision's u_b != 0 branch.  Within the storage formats'
    rounding of the oracle (FP64) at every checkpoint to t = 300."""
    w = W.vortex_512x256(nx=256, ny=128)
    worst = _run_pair(256, 128, w.tau, w.fields, [1, 10, 100, 300], store, tol, w.u_ref, m0=w.m0,
                      ubase=(0.1, 0.0))
    print(f"  worst {store}: e_rho={worst[0]:.3e} e_u={worst[1]:.3e}", flush=True)


def test_vortex512x256_fp32_rest_base_error_report():
    """Same run with deviations about the rest state (f_i - w_i rho0): the mean flow then sits in
    the stored values and fp32 rounding of it drifts coherently; reported, with a sanity bound."""
    w = W.vortex_512x256()
    _run_pair(w.nx, w.ny, w.tau, w.fields, [100, 1000], "f32", 3e-4, w.u_ref, m0=w.m0)


def test_fp32_ragged_with_farfield():
    f = W.lamb_oseen(131, 77, 60.0, 40.0, 8.0, W.swirl_amplitude(0.02), (0.08, 0.02))
    _run_pair(131, 77, 0.53, f, [1, 50, 300], "f32", 1e-5, 0.08, beta=0.2, m0=(1.0, 0.08, 0.02),
              ubase=(0.08, 0.02))


def test_step_zero_and_time():
    w = W.pulse_128(32, 32)
    g = _lattice(nx=32, ny=32, tau=0.6, fields=w.fields, store="f64")
    before = g.populations().cpu().numpy()
    g.step(0)
    assert g.t == 0
    assert np.array_equal(before, g.populations().cpu().numpy())
    g.step(3)
    assert g.t == 3


def test_init_populations_are_equilibrium():
    """Right after init the stored set is g^eq of the initial fields (oracle's init)."""
    f = W.lamb_oseen(40, 30, 20.0, 15.0, 5.0, 0.05, (0.05, 0.01))
    g = _lattice(nx=40, ny=30, tau=0.6, fields=f, store="f64")
    o = oracle.Lattice(40, 30, 0.6, *f)
    assert np.abs(g.populations().cpu().numpy() - o.g).max() < 1e-17
    h = _lattice(nx=40, ny=30, tau=0.6, fields=f, store="f64", ubase=(0.05, 0.01))
    assert np.abs(h.populations().cpu().numpy() - o.g).max() < 1e-16


def test_all_tiles_bitwise_identical():
    """Every bulk tile shape computes the same per-node arithmetic: identical bits."""
    from paper_2005_08674_amd import lbm
    f = W.gaussian_pulses(203, 77, [(1e-3, 6.0, 90.0, 40.0)], u0=(0.02, 0.0))
    ref = None
    for store in ("f64", "f32", "f16", "bf16"):
        ref = None
        for tile in range(lbm.lbm_tile_count()):
            g = _lattice(nx=203, ny=77, tau=0.6, fields=f, store=store)
            lbm.lbm_set_tile(g.ctx, tile)
            g.step(5)
            pops = g.populations().cpu().numpy()
            if ref is None:
                ref = pops
            else:
                assert np.array_equal(pops, ref), (store, tile)
            g.close()


def test_run_twice_identical():
    w = W.vortex_512x256(nx=256, ny=128)
    a = _lattice(nx=256, ny=128, tau=0.55, fields=w.fields, store="f32", m0=w.m0)
    b = _lattice(nx=256, ny=128, tau=0.55, fields=w.fields, store="f32", m0=w.m0)
    a.step(200)
    b.step(100)
    b.step(100)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())


def test_set_get_populations_roundtrip_and_continue():
    """Checkpoint/restore: copying the state into a new context and continuing is bitwise equal."""
    w = W.pulse_128(64, 48)
    a = _lattice(nx=64, ny=48, tau=0.6, fields=w.fields, store="f64")
    a.step(20)
    snap = a.populations()
    b = _lattice(nx=64, ny=48, tau=0.6, fields=w.fields, store="f64")
    b.set_populations(snap)
    a.step(30)
    b.step(30)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())


def test_full_size_4096_fp32_against_oracle():
    """4096^2 fp32 (the HBM workload) in the tuned launch shape: 10 steps vs the oracle, every node."""
    w = W.pulses_4096()
    g = _lattice(nx=w.nx, ny=w.ny, tau=w.tau, fields=w.fields, store="f32")
    g.autotune(reps=3)
    g.step(10)
    gm = g.moments_np()
    g.close()
    o = oracle.Lattice(w.nx, w.ny, w.tau, *w.fields)
    o.step(10)
    er, eu = _errors(gm, o.moments(), 1.0, w.u_ref)
    print(f"\n[parity 4096^2 fp32] e_rho={er:.3e} e_u={eu:.3e}", flush=True)
    assert er <= 1e-5 and eu <= 1e-5


def test_nonfinite_detected():
    f = W.uniform(16, 16)
    g = _lattice(nx=16, ny=16, tau=0.6, fields=f, store="f32")
    assert g.check_finite()
    pops = g.populations()
    pops[3, 5, 5] = float("nan")
    g.set_populations(pops)
    assert not g.check_finite()


def test_overlap_matches_serial():
    """Edge kernel on the side stream (overlapped) or after the bulk kernel: identical bits."""
    from paper_2005_08674_amd import lbm
    w = W.vortex_512x256(nx=192, ny=96)
    a = _lattice(nx=192, ny=96, tau=0.55, fields=w.fields, store="f32", m0=w.m0, ubase=(0.1, 0.0))
    b = _lattice(nx=192, ny=96, tau=0.55, fields=w.fields, store="f32", m0=w.m0, ubase=(0.1, 0.0))
    lbm.lbm_set_overlap(a.ctx, True)
    lbm.lbm_set_overlap(b.ctx, False)
    for n in (1, 5, 37):
        a.step(n)
        b.step(n)
        assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())


def test_kernel_timing_counts_launches():
    """Fused step launches count as bulk launches; separate launches count both kernels."""
    from paper_2005_08674_amd import lbm
    w = W.pulse_128(256, 256)
    g = _lattice(nx=256, ny=256, tau=0.6, fields=w.fields, store="f32")
    lbm.lbm_enable_timing(g.ctx, True)
    g.step(25)
    bm, bn, em, en = lbm.lbm_kernel_times(g.ctx)
    assert bn == 25 and en == 0 and bm > 0
    b, n = lbm.lbm_bulk_traffic(g.ctx)
    assert b == 72 and n == 256 * 256
    lbm.lbm_set_fused(g.ctx, False)
    g.step(25)
    bm, bn, em, en = lbm.lbm_kernel_times(g.ctx)
    assert bn == 25 and en == 25 and bm > 0 and em > 0
    lbm.lbm_enable_timing(g.ctx, False)
    b, n = lbm.lbm_bulk_traffic(g.ctx)
    assert b == 72 and n == 254 * 254


@pytest.mark.parametrize("store", ["f64", "f32", "f16", "bf16"])
def test_fused_step_equals_separate_launches(store):
    """One launch per step (edge segments + bulk tiles) gives the bits of the two separate launches,
    for every tile shape, on ragged lattices with mixed edges."""
    from paper_2005_08674_amd import lbm
    cases = [dict(nx=203, ny=77), dict(nx=65, ny=130, bc=(0, 0, 1, 1)), dict(nx=3, ny=3), dict(nx=130, ny=4, bc=(1, 1, 0, 0))]
    for kw in cases:
        f = W.gaussian_pulses(kw["nx"], kw["ny"], [(1e-3, 4.0, kw["nx"] / 3, kw["ny"] / 2)], u0=(0.02, -0.01))
        for tile in range(lbm.lbm_tile_count()):
            a = _lattice(tau=0.58, fields=f, store=store, beta=0.2, m0=(1.0001, 0.02, -0.01), **kw)
            b = _lattice(tau=0.58, fields=f, store=store, beta=0.2, m0=(1.0001, 0.02, -0.01), **kw)
            lbm.lbm_set_tile(a.ctx, tile)
            lbm.lbm_set_tile(b.ctx, tile)
            lbm.lbm_set_fused(b.ctx, False)
            a.step(6)
            b.step(6)
            assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy()), (store, kw, tile)
            a.close()
            b.close()


@pytest.mark.parametrize("nbytes", [16, 4096 + 7, 3 * 1000003])
def test_stream_copy(nbytes):
    from paper_2005_08674_amd import lbm
    src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    lbm.lbm_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)


def test_storage_error_against_fp64_at_4096():
    """pulses4096 with FP32, FP16 and BF16 deviation storage (FP32 arithmetic) against the same run in
    FP64 (itself parity-checked against the oracle), each in its tuned launch (three steps per launch
    at this size), at t = 100, 500, 1000, 2000: the error each storage
    format adds, stated per run.  Bounds: FP32 1e-5 (the parity bar); FP16 and BF16, whose rounding is
    2^-11 and 2^-8 of the stored deviation, 2e-2 and 1e-1 of U_ref."""
    from paper_2005_08674_amd import autotune
    w = W.pulses_4096()
    runs = {s: _lattice(nx=w.nx, ny=w.ny, tau=w.tau, fields=w.fields, store=s) for s in ("f64", "f32", "f16", "bf16")}
    for s, g in runs.items():
        # every format in the launch the benchmark times (the cached autotuner choice)
        name = autotune.apply(g, s)
        if name is None:
            autotune.tune(g, s, reps=3, path=None)
        print(f"[storage 4096^2] {s}: {name}", flush=True)
    bounds = {"f32": 1e-5, "f16": 2e-2, "bf16": 1e-1}
    t = 0
    for t_next in (100, 500, 1000, 2000):
        for g in runs.values():
            g.step(t_next - t)
        t = t_next
        ref = runs["f64"].moments()
        for s in ("f32", "f16", "bf16"):
            m = runs[s].moments()
            er = float((m[0] - ref[0]).abs().max()) / 1.0
            eu = max(float((m[1] - ref[1]).abs().max()), float((m[2] - ref[2]).abs().max())) / w.u_ref
            print(f"[storage {s} vs fp64, 4096^2] t={t}: e_rho={er:.3e} e_u={eu:.3e}", flush=True)
            assert er <= bounds[s] and eu <= bounds[s], (s, t, er, eu)
        del ref
    for g in runs.values():
        g.close()
