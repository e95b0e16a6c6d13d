#!/usr/bin/env python3
"""Throughput of the D2Q9 BGK + NSBC sweep on one MI355X.

One step = one lbm_step(1): one fused launch whose first blocks run the NSBC
edge/corner segments over the perimeter and the rest the bulk collide-stream
tiles over the interior.  Workload: 4096 x 4096
lattice, tau 0.51, 8 seeded Gaussian pulses (amplitude U[1e-4, 1e-3],
half-width U[4, 16]), NSBC on all four edges, populations stored as FP32
deviations f_i - w_i rho0 (the headline), plus FP16/BF16-deviation and FP64
variants.  Inputs are resident in HBM before timing starts.  Further
variants: the 256-lattice batched ensemble in one graph launch, and the
2048^2 vortex + pulse case run with plain NSBC (FP32, FP16 storage) and with
the learned closure, each with its reflection coefficient against an 8192^2
reference.

Prints ONE JSON line (rank 0): metric/value (MLUPS), ms_per_step, the step
kernel's roofline fraction from HIP-event durations measured over the same K
steps, and the CPU fp64 oracle timed on a bounded sample of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS D2Q9+NSBC (FP32 vs FP16 store, MLP closure); % HBM peak; reflection"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def copy_ceiling(torch, nbytes, reps=20):
    """GB/s of the library's plain copy kernel moving nbytes in + nbytes out (median of reps)."""
    from paper_2005_08674_amd import lbm
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    lbm.lbm_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, stream.cuda_stream)
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        lbm.lbm_stream_copy(src.data_ptr(), dst.data_ptr(), nbytes, stream.cuda_stream)
        b.record(stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    ts.sort()
    ms = ts[len(ts) // 2]
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9, ms


MRT_RATES = (1.9, 1.9, 1.9)   # omega_e, omega_eps, omega_q of the paper's test case 1 (Sec. 6)


def run_store(torch, W, store, steps, warmup, tune_reps=5, size=4096, serial_check=False, tile=None, retune=False,
              mrt=None):
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice

    w = W.pulses_4096(n=size)
    lat = Lattice(w.nx, w.ny, w.tau, w.fields, store=store, mrt=mrt)
    from paper_2005_08674_amd import autotune
    if tile:
        # a single-step tile name, or a multi-step shape name ("2step:..." or "3step:...")
        names = [lbm.lbm_tile_describe(i) for i in range(lbm.lbm_tile_count())]
        twos = [lbm.lbm_two_step_describe(i) for i in range(lbm.lbm_two_step_count())]
        if tile in twos:
            lbm.lbm_set_two_step(lat.ctx, twos.index(tile))
        else:
            lbm.lbm_set_tile(lat.ctx, names.index(tile))
        tile_name = tile
        log(f"[{store}] launch shape fixed to {tile}")
    else:
        tile_name = None if retune else autotune.apply(lat, store)
        if tile_name:
            log(f"[{store}] launch shape from the autotuner cache: {tile_name}")
        else:
            e = autotune.tune(lat, store, reps=tune_reps, path=None)
            tile_name = e["tile"] if not e["two_step"] else f"{e['tile']} | {e['two_step']}"
            log(f"[{store}] autotune -> {tile_name}; "
                + ", ".join(f"{n}={t:.4f}" for n, t in e["candidates"].items())
                + "; multi-step (ms per step): "
                + ", ".join(f"{n}={t:.4f}" for n, t in e.get("two_step_candidates", {}).items()))
    two_step = lbm.lbm_get_two_step(lat.ctx) >= 0
    lat.step(warmup)
    stream = lat.stream
    torch.cuda.synchronize()
    if serial_check:
        for ov in (True, False):
            lbm.lbm_set_overlap(lat.ctx, ov)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            lat.step(100)
            b.record(stream)
            torch.cuda.synchronize()
            log(f"[{store}] overlap={ov}" + (" (separate single-step launches)" if ov else "") + f": {a.elapsed_time(b) / 100:.5f} ms/step")
    # Timed region: K steps, bracketed by synchronisation, no instrumentation.
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = e0.elapsed_time(e1)
    # The same K steps again with every kernel launch bracketed by HIP events
    # on the stream it runs on: per-launch durations for the roofline.  A
    # launch is either the two-step sweep (two steps of every node) or the
    # fused single-step launch (edge segments + bulk tiles), which the timing
    # counts as the step's bulk launch.
    lbm.lbm_enable_timing(lat.ctx, True)
    lat.step(steps)
    two_ms, two_n = lbm.lbm_two_step_times(lat.ctx)
    bulk_ms, bulk_n, edge_ms, edge_n = lbm.lbm_kernel_times(lat.ctx)
    lbm.lbm_enable_timing(lat.ctx, False)
    bpn, nodes_launch = lbm.lbm_bulk_traffic(lat.ctx)
    steps_per_launch = 1
    kernel_shape = lbm.lbm_tile_describe(lbm.lbm_get_tile(lat.ctx))
    if two_step and two_n > 0:
        kernel_shape = lbm.lbm_two_step_describe(lbm.lbm_get_two_step(lat.ctx))
        # algorithmic bytes per node-step (2 x 9 x s) x the node-steps one launch advances
        bulk_ms, bulk_n = two_ms, two_n
        nodes_launch = w.nx * w.ny
        steps_per_launch = lbm.lbm_two_step_steps(lbm.lbm_get_two_step(lat.ctx))
    ok = lat.check_finite()
    nodes = w.nx * w.ny
    out = {
        "store": store,
        "tile": tile_name,
        "ms_per_step": ms / steps,
        "wall_s": t_wall,
        "mlups": nodes * steps / (ms * 1e-3) / 1e6,
        "kernel": ("two-step sweep (t -> t + 2, level t + 1 in LDS)" if steps_per_launch == 2 else
                   "three-step sweep (t -> t + 3, levels t + 1 and t + 2 in LDS)" if steps_per_launch == 3 else
                   "fused step launch (edge segments + bulk tiles)"),
        "kernel_avg_ms": bulk_ms / max(bulk_n, 1),
        "separate_edge_launches": edge_n,
        "bytes_per_node": bpn,
        "nodes_per_launch": nodes_launch,
        "steps_per_launch": steps_per_launch,
        "kernel_shape": kernel_shape,
        "finite": bool(ok),
        "workload": w,
    }
    # The bytes one launch must move: one read and one write of every node's 9 populations (2 x 9 x s
    # per node), whatever number of steps the launch advances -- a multi-step launch keeps its
    # intermediate levels on chip, so this one pass is its HBM floor.  The single-step-equivalent
    # rate (2 x 9 x s per node and step advanced) is kept beside it under its own name.
    dur = out["kernel_avg_ms"] * 1e-3
    achieved = bpn * nodes_launch / dur / 1e9
    out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                       "step_equivalent_GBs": round(bpn * nodes_launch * steps_per_launch / dur / 1e9, 1)}
    lat.close()
    return out


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "multistep_pulses4096_f32_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2005_08674_amd", "csrc", f)
                  for f in ("lbm_kernels.hip", "lbm_twostep.hip", "lbm_device.h", "lbm_sweep.h", "lbm_twostep_lds.h",
                            "lbm_threestep.h", "lbm_march.hip")]


def kernel_source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(tile: str):
    """HBM bytes per launch of the dominant kernel measured with rocprofv3 counters (profiles/), or
    None when the record is missing, was taken with another launch shape, or the kernel sources
    changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel_source_sha256") != kernel_source_sha() or rec.get("tile") != tile:
        return None
    try:
        return float(rec["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


COUNTERS_FILE = os.path.join(ROOT, "profiles", "multistep_pulses4096_f32_sq_counters.md")


def recorded_counters(tile: str):
    """The dominant kernel's SQ counter summary (VALU issue fraction and the like) from profiles/,
    when it was taken on the current kernel sources and this launch shape; else None."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    rec = {}
    with open(COUNTERS_FILE) as f:
        for line in f:
            line = line.strip().lstrip("-* ").strip()
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip().strip("`")] = v.strip().strip("`")
    if rec.get("kernel_source_sha256") != kernel_source_sha() or rec.get("tile") != tile:
        return None
    out = {}
    for k in ("valu_issue_frac", "wave_wait_frac", "valu_insts_per_node_update", "node_updates_per_output_node"):
        try:
            out[k] = float(rec[k])
        except (KeyError, ValueError):
            pass
    return out or None


def run_tc1(torch, W):
    """Test case 1 of Sec. 6 (128^2 plane wave at 60 degrees, MRT at tau = 1/2, rates 1.9, NSBC gamma 0.6):
    the acoustic energy left in the domain after the wave has crossed it, relative to the wave's own
    (the library's fp64 energy reduction), for FP32 and FP64 storage."""
    from paper_2005_08674_amd.lattice import Lattice

    w = W.plane_wave_tc1()
    out = {"workload": f"{w.name}: {w.nx}x{w.ny}, theta 60 deg, zeta 0.01, lambda {w.nx / 32:g}, tau 0.5, "
                       f"MRT rates {w.mrt}, NSBC gamma 0.6 beta 0", "steps": w.steps}
    for store in ("f32", "f64"):
        lat = Lattice(w.nx, w.ny, w.tau, w.fields, store=store, mrt=w.mrt)
        e0 = float(lat.energy().item())
        lat.step(w.steps)
        out[f"residual_energy_{store}"] = float(lat.energy().item()) / e0
        out[f"finite_{store}"] = bool(lat.check_finite())
        lat.close()
    return out


def run_tc2(torch, W, every=50):
    """Test case 2 of Sec. 7 (128^2 convected vortex: velocity inlet left, NSBC right, periodic bottom and
    top, MRT 1.4/1.2, Re 1000): R_E against a lattice 4x wider to the right (the window's continuation,
    the library's fp64 energy reduction every `every` steps) and the transverse velocity left after the
    vortex has gone, for NSBC (gamma 0.6) and, for comparison, gamma 0."""
    from paper_2005_08674_amd.lattice import Lattice

    w = W.convected_vortex_tc2()
    wr = W.convected_vortex_tc2(nx=4 * w.nx)
    out = {"workload": f"{w.name}: {w.nx}x{w.ny}, Lamb-Oseen u0 0.1, U_v 0.05, R_c 20, tau {w.tau:.4f}, MRT rates "
                       f"{w.mrt}, inlet u_w {w.uw}, NSBC right (beta 0), periodic bottom/top; reference "
                       f"{wr.nx}x{wr.ny}", "steps": w.steps, "energy_every": every}

    def lat(wk, gamma, store):
        return Lattice(wk.nx, wk.ny, wk.tau, wk.fields, store=store, bc=wk.bc, gamma=gamma, m0=wk.m0, mrt=wk.mrt,
                       uw=wk.uw, ubase=wk.uw)

    v0 = float(np.abs(w.fields[2]).max())
    for store in ("f32", "f64"):
        ref = lat(wr, 0.6, store)
        for gamma in (0.6, 0.0):
            test = lat(w, gamma, store)
            e0 = float(test.energy(ux_ref=w.uw[0], uy_ref=w.uw[1]).item())
            series = torch.zeros(w.steps // every + 1, dtype=torch.float64, device=test.device)
            r = lat(wr, 0.6, store) if gamma != 0.6 else ref
            for k in range(series.numel()):
                test.energy(ref=r, out=series[k:k + 1])
                if k + 1 < series.numel():
                    test.step(every)
                    r.step(every)
            v = float(np.abs(test.moments_np()[2]).max())
            out[f"{store}_gamma{gamma}"] = {"R_E": float(series.max().item()) / e0, "vmax_final_rel": v / v0,
                                            "finite": bool(test.check_finite())}
            test.close()
            if r is not ref:
                r.close()
        ref.close()
    return out


def run_3d(torch, W, steps, n=256, q=19):
    """The D3Q19 (q = 19) or D3Q27 (q = 27) sweep on an n^3 lattice (8 seeded pulses, tau 0.55, NSBC on all
    six faces), FP32, FP64, FP16 and BF16 storage: MLUPS over `steps` steps in one timed region after the
    shape autotuner, and the algorithmic-bytes fraction of the HBM peak (2 x q x s bytes per node-step,
    one launch per step)."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice3d import Lattice3D

    fields, _ = W.pulses_3d(n)
    out = {"workload": f"pulses3d{n}: {n}^3 D3Q{q} BGK tau 0.55, 8 seeded Gaussian pulses, NSBC (gamma 0.6, "
                       "beta 0) on 6 faces", "steps": steps}
    for store, s in (("f32", 4), ("f64", 8), ("f16", 2), ("bf16", 2)):
        lat = Lattice3D(n, n, n, 0.55, fields, store=store, q=q)
        best, times = lat.autotune(reps=5)
        lat.step(10)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(lat.stream)
        lat.step(steps)
        b.record(lat.stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        ok = all(np.isfinite(m).all() for m in lat.moments())
        lat.close()
        gbs = 2 * q * s * n ** 3 / (ms * 1e-3) / 1e9
        out[store] = {"mlups": round(n ** 3 / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 5),
                      "shape": lbm.lbm3d_shape_describe(best),
                      "shape_ms": {lbm.lbm3d_shape_describe(i): round(t, 5) for i, t in enumerate(times)},
                      "bytes_per_node": 2 * q * s, "achieved_GBs": round(gbs, 1),
                      "roofline_frac": round(gbs / HBM_PEAK_GBS, 4), "finite": bool(ok)}
    return out


def run_ensemble(torch, W, steps, count=256, seed=4):
    """The batched-ensemble workload: `count` lattices with sides U{64..512}, tau U[0.52, 0.8], pulse or
    vortex, FP32 storage; `steps` steps in ONE graph launch (captured beforehand)."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.ensemble import Ensemble, member_params
    ms = W.ensemble_members(count, seed=seed)
    members = [member_params(m.nx, m.ny, m.tau, store="f32",
                             ubase=(m.params["u0"] if m.kind == "vortex" else (0.0, 0.0))) for m in ms]
    ens = Ensemble(members, [W.member_fields(m) for m in ms])
    for k, m in enumerate(ms):
        ens.set_farfield(k, 0.0, *W.member_m0(m))
    best, times = ens.autotune(reps=5)
    shape = lbm.lbm_ens_shape_describe(best)
    # the multi-step sweep when it beats single steps per step
    b2, t2 = ens.autotune_two_step(reps=5)
    two = None
    if t2[b2] < times[best]:
        two = lbm.lbm_two_step_describe(b2)
    else:
        ens.set_two_step(-1)
    nodes, nb, ne = ens.info()
    ens.step_graph(steps)  # capture, instantiate, first launch (untimed)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(ens.stream)
    ens.step_graph(steps)
    b.record(ens.stream)
    torch.cuda.synchronize()
    ms_ = a.elapsed_time(b)
    ens.close()
    bulk_nodes = sum((m.nx - 2) * (m.ny - 2) for m in ms)
    return {"mlups": round(nodes * steps / (ms_ * 1e-3) / 1e6, 1), "ms_per_step": round(ms_ / steps, 5),
            "members": count, "nodes": nodes, "steps_per_graph_launch": steps, "shape": shape, "two_step": two,
            "two_step_ms_by_shape": {lbm.lbm_two_step_describe(i): round(t, 5) for i, t in enumerate(t2)},
            "bulk_blocks": nb, "edge_blocks": ne, "bulk_ms_by_shape": {lbm.lbm_ens_shape_describe(i): round(t, 5)
                                                                      for i, t in enumerate(times)},
            "step_GBs_algorithmic": round(72 * nodes / (ms_ / steps * 1e-3) / 1e9, 1)}


CLOSURE_NET = os.path.join(ROOT, "paper_2005_08674_amd", "data", "closure_c4.npz")


def run_c5(torch, W, steps, every=50, timing_steps=1000):
    """Vortex + pulse on a 2048^2 lattice (tau 0.55, u0 = (0.1, 0)): plain NSBC and the learned closure,
    each with FP32 and FP16 deviation storage, each with its MLUPS (test lattice alone) and its
    reflection coefficient R_E against an 8192^2 FP32 reference over `steps` steps."""
    from paper_2005_08674_amd import lbm
    from paper_2005_08674_amd.lattice import Lattice
    from paper_2005_08674_amd.reflection import ReflectionRun
    w = W.vortex_pulse_2048()
    ex = w.extra
    u0 = (0.1, 0.0)
    n = w.nx

    def field(x, y):
        dv, ux, uy = W.lamb_oseen_xy(x, y, ex["x0"], ex["y0"], ex["rc"], ex["uv"], u0)
        dp = 1e-3 * np.exp(-np.log(2.0) * ((x - n / 2.0) ** 2 + (y - n / 2.0) ** 2) / 64.0)
        return dv + dp, ux, uy

    blob, net_note = None, None
    if os.path.exists(CLOSURE_NET):
        from paper_2005_08674_amd.closure import Trainer
        tr = Trainer.load(CLOSURE_NET)
        blob = tr.export()
        net_note = {k: v for k, v in tr.meta.items()}
    out = {"workload": f"vortexpulse{n}: {n}x{n} tau 0.55, u0 (0.1, 0), Lamb-Oseen vortex (R_c 12, max swirl "
                       f"0.02) at ({ex['x0']:.1f}, {ex['y0']:.1f}) + pulse (1e-3, HWHM 8) at the centre; NSBC "
                       f"gamma 0.6, beta 0, m0 (1, 0.1, 0); reference {4 * n}^2 FP32",
           "steps": steps, "energy_every": every}
    runs = [("nsbc_f32", "f32", None), ("nsbc_f16", "f16", None)]
    if blob is not None:
        runs += [("closure_f32", "f32", blob), ("closure_f16", "f16", blob)]
    def use(lat, choice):
        kind, k = choice
        if kind == "multi":
            lbm.lbm_set_two_step(lat.ctx, k)
            return lbm.lbm_two_step_describe(k)
        lbm.lbm_set_two_step(lat.ctx, -1)
        lbm.lbm_set_tile(lat.ctx, k)
        return lbm.lbm_tile_describe(k)

    def fastest(lat, reps=5):
        """Tune the launch on `lat` (the library's tuners time consecutive steps from a saved state);
        keep the multi-step sweep when it beats single steps per step.  Returns the choice."""
        best, times = lbm.lbm_autotune(lat.ctx, reps)
        b2, t2 = lbm.lbm_autotune_two_step(lat.ctx, reps)
        return ("multi", b2) if t2[b2] < times[best] else ("single", best)

    def closure_overlap(lat, steps=100):
        """Time closure steps with the edge kernel on the lattice's stream and on a second stream
        overlapping the bulk kernel (same results); keep the faster."""
        t = {}
        for ov in (False, True):
            lbm.lbm_set_overlap(lat.ctx, ov)
            lat.step(4)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(lat.stream)
            lat.step(steps)
            b.record(lat.stream)
            torch.cuda.synchronize()
            t[ov] = a.elapsed_time(b)
        best = t[True] < t[False]
        lbm.lbm_set_overlap(lat.ctx, best)
        return best

    for name, store, net in runs:
        g = Lattice(n, n, w.tau, w.fields, store=store, m0=(1.0, 0.1, 0.0), ubase=u0)
        if net is not None:
            lbm.lbm_set_closure(g.ctx, net.data_ptr(), 1)
        # the same tuning for both: with the closure the three-step shapes carry the network
        choice = fastest(g)
        launch = use(g, choice)
        overlap = False
        if net is not None:
            if choice[0] == "single":
                overlap = closure_overlap(g)
                launch += (" + edge (closure) kernel on a second stream beside the bulk kernel" if overlap
                           else " + edge (closure) kernel after the bulk kernel")
            else:
                launch += " (edge tiles with the network in a kernel on a second stream beside the inner tiles)"
        g.step(20)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(g.stream)
        g.step(timing_steps)
        b.record(g.stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        g.close()
        rr = ReflectionRun(field, n, n, w.tau, scale=4, store=store, ref_store="f32", u0=u0, ubase=u0,
                           closure=net)
        use(rr.test, choice)  # the same lattice size and parameters as the timing lattice
        if overlap:
            lbm.lbm_set_overlap(rr.test.ctx, True)
        use(rr.ref, fastest(rr.ref))
        res = rr.run(steps, every=every, respect_clean_time=True)
        finite = rr.test.check_finite()
        rr.close()
        out[name] = {"mlups": round(n * n * timing_steps / (ms * 1e-3) / 1e6, 1), "launch": launch,
                     "ms_per_step": round(ms / timing_steps, 5), "R_E": float(res["R_E"]),
                     "R_E_final": float(res["series"][-1]), "R_E_at_most_1e-3": bool(res["R_E"] <= 1e-3),
                     "horizon": res["horizon"], "finite": bool(finite)}
    if net_note is not None:
        out["closure_net"] = {"file": os.path.relpath(CLOSURE_NET, ROOT), **net_note}
    return out


# algorithmic flops per training sample of the closure network 96 -> 64 -> 64 -> 3:
# forward 2 (96*64 + 64*64 + 64*3); backward dW1, dW2, dW3 and the input
# gradients of layers 2 and 3
MLP_FWD_FLOPS = 2 * (96 * 64 + 64 * 64 + 64 * 3)
MLP_TRAIN_FLOPS = MLP_FWD_FLOPS + 2 * (96 * 64 + 64 * 64 + 64 * 3) + 2 * (64 * 64 + 64 * 3)
BF16_PEAK_TFLOPS = 2500.0


def run_training(torch, steps=300, batches=(4096, 65536), nsamples=1 << 19):
    """Closure training throughput: Adam steps on minibatches of BF16 inputs (random normalised
    samples; the cost does not depend on their values), timed with events.  4096 is the batch the
    training uses (64 blocks of 64 rows: a quarter of the chip, latency-bound); 65536 fills it."""
    from paper_2005_08674_amd.closure import Trainer
    g = torch.Generator(device="cuda").manual_seed(7)
    x = torch.randn((nsamples, 96), device="cuda", generator=g).to(torch.bfloat16)
    t = torch.randn((nsamples, 3), device="cuda", generator=g)
    out = {"flops_per_sample": MLP_TRAIN_FLOPS}
    for batch in batches:
        tr = Trainer(max_batch=batch)
        rows = torch.randint(0, nsamples, (steps, batch), device="cuda", dtype=torch.int32, generator=g)
        for k in range(5):
            tr.train_step(x, t, 1e-4, rows=rows[k])
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(tr.stream)
        for k in range(steps):
            tr.train_step(x, t, 1e-4, rows=rows[k])
        b.record(tr.stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        sps = batch / (ms * 1e-3)
        tflops = sps * MLP_TRAIN_FLOPS / 1e12
        out[f"batch{batch}"] = {
            "ms_per_step": round(ms, 5), "samples_per_s": round(sps, 1),
            "roofline": {"bound": "mfma", "achieved": round(tflops, 3), "peak": BF16_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tflops / BF16_PEAK_TFLOPS, 6)}}
        tr.close()
        del rows
    return out


CPU_RUNS = [
    # (name, workload factory, steps with one thread, steps with all threads)
    ("pulse128", "pulse_128", 1000, 1000),
    ("vortex512x256", "vortex_512x256", 200, 1000),
    ("pulses4096", "pulses_4096", 3, 20),
]

_CPU_CHILD = r"""
import json, sys, time
sys.path.insert(0, {root!r})
import oracle
from paper_2005_08674_amd import workloads as W
w = getattr(W, {factory!r})()
o = oracle.Lattice(w.nx, w.ny, w.tau, *w.fields, m0=getattr(w, "m0", None) or (1.0, 0.0, 0.0))
o.step(1)
t0 = time.perf_counter()
o.step({steps})
dt = time.perf_counter() - t0
print(json.dumps({{"nodes": w.nx * w.ny, "steps": {steps}, "s": dt, "threads": oracle.num_threads()}}))
"""


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W, w):
    """The fp64 oracle (plain C, OpenMP over rows) timed on the host: the 128^2 pulse in full (1000
    steps), the 512x256 vortex and the 4096^2 pulses for a bounded number of steps, each with one
    thread and with every thread the process may use (OMP_NUM_THREADS, else the CPU count), each in
    a child process, one untimed step and lattice set-up excluded.  `value` is the 4096^2 figure with
    all threads, the workload `value` of this line is measured on."""
    import subprocess
    nproc = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    runs = []
    for threads in (1, nproc):
        for name, factory, s1, sn in CPU_RUNS:
            steps = s1 if threads == 1 else sn
            env = {**os.environ, "OMP_NUM_THREADS": str(threads)}
            r = subprocess.run([sys.executable, "-c", _CPU_CHILD.format(root=ROOT, factory=factory, steps=steps)],
                               env=env, capture_output=True, text=True, timeout=600)
            if r.returncode != 0:
                log(f"[cpu_baseline] {name} x{threads} failed: {r.stderr[-500:]}")
                continue
            d = json.loads(r.stdout.strip().splitlines()[-1])
            runs.append({"workload": name, "threads": d["threads"], "steps": d["steps"], "seconds": round(d["s"], 3),
                         "MLUPS": round(d["nodes"] * d["steps"] / d["s"] / 1e6, 3)})
            log(f"[cpu_baseline] {runs[-1]}")
    head = [r for r in runs if r["workload"] == "pulses4096" and r["threads"] == nproc]
    return {"value": head[0]["MLUPS"] if head else None, "unit": "MLUPS",
            "cores": head[0]["threads"] if head else nproc, "kind": "oracle",
            "sample": f"{w.nx}x{w.ny} pulse workload, {CPU_RUNS[2][3]} fp64 oracle steps with {nproc} threads "
                      "(set-up and one step excluded); runs lists the other samples",
            "cpu_model": cpu_model(), "runs": runs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--variants", default="f16,bf16,f64,mrt_f32,mrt_f16",
                    help="extra variants: storage formats, mrt_<store> for the MRT collision ('' for none)")
    ap.add_argument("--tc1", type=int, default=1, help="0 skips the paper's test cases 1 and 2")
    ap.add_argument("--variant-steps", type=int, default=500)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-reps", type=int, default=5)
    ap.add_argument("--no-copy-ref", action="store_true")
    ap.add_argument("--tile", default=None, help="fix the FP32 bulk tile by name instead of autotuning")
    ap.add_argument("--retune", action="store_true", help="ignore the autotuner cache and re-time all tiles")
    ap.add_argument("--ensemble-steps", type=int, default=2000, help="0 skips the ensemble variant")
    ap.add_argument("--c5-steps", type=int, default=6000, help="0 skips the 2048^2 vortex+pulse reflection runs")
    ap.add_argument("--train-steps", type=int, default=300, help="0 skips the closure-training throughput run")
    ap.add_argument("--d3-steps", type=int, default=200, help="0 skips the D3Q19 and D3Q27 256^3 runs")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2005_08674_amd import lbm, workloads as W
    lbm.load()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)

    main_run = run_store(torch, W, "f32", args.steps, args.warmup, tune_reps=args.tune_reps, size=args.size,
                         serial_check=True, tile=args.tile, retune=args.retune)
    variants = {}
    for st in [s for s in args.variants.split(",") if s]:
        mrt = MRT_RATES if st.startswith("mrt_") else None
        r = run_store(torch, W, st[4:] if mrt else st, args.variant_steps, min(args.warmup, 20),
                      tune_reps=args.tune_reps, size=args.size, retune=args.retune, mrt=mrt)
        variants[st] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 5),
                        "kernel_avg_ms": round(r["kernel_avg_ms"], 5), "steps_per_launch": r["steps_per_launch"],
                        "tile": r["tile"],
                        "roofline_frac": r["roofline"]["frac"], "achieved_GBs": r["roofline"]["achieved"],
                        "steps": args.variant_steps, "finite": r["finite"]}
    if args.tc1:
        variants["planewave128_tc1"] = run_tc1(torch, W)
        variants["convectedvortex128_tc2"] = run_tc2(torch, W)
    if args.ensemble_steps > 0:
        variants["ensemble256_f32"] = run_ensemble(torch, W, args.ensemble_steps)
    if args.d3_steps > 0:
        variants["pulses3d256_d3q19"] = run_3d(torch, W, args.d3_steps)
        variants["pulses3d256_d3q27"] = run_3d(torch, W, args.d3_steps, q=27)
    if args.c5_steps > 0:
        variants["vortexpulse2048_reflection"] = run_c5(torch, W, args.c5_steps)
    if args.train_steps > 0:
        variants["closure_training"] = run_training(torch, steps=args.train_steps)
    w = main_run["workload"]
    traffic = recorded_traffic(main_run["kernel_shape"])
    if traffic is not None:
        main_run["roofline"]["traffic"] = traffic
        # the counters' bytes over the same launch duration: the HBM bandwidth the kernel really draws
        main_run["roofline"]["traffic_GBs"] = round(traffic / (main_run["kernel_avg_ms"] * 1e-3) / 1e9, 1)
    main_run["roofline"]["basis"] = (
        f"achieved = the bytes one launch must move, one read and one write of the state "
        f"({main_run['bytes_per_node']} B per node = 2 x 9 x 4 B, x {main_run['nodes_per_launch']} nodes), "
        f"over the kernel's average launch duration ({main_run['kernel_avg_ms']:.5f} ms, HIP events on its stream); "
        f"the launch advances {main_run['steps_per_launch']} step(s), keeping intermediate levels on chip; "
        "step_equivalent_GBs counts 2 x 9 x 4 B per node and step advanced instead")
    sq = recorded_counters(main_run["kernel_shape"])
    if sq:
        main_run["roofline"]["counters"] = sq
    line = {
        "metric": METRIC,
        "value": round(main_run["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.nx}x{w.ny} D2Q9 BGK tau {w.tau}, 8 seeded Gaussian pulses, "
                               "NSBC (gamma 0.6, beta 0) on 4 edges, FP32 deviation storage, FP32 compute",
                   "nx": w.nx, "ny": w.ny, "store": "f32", "tile": main_run["tile"],
                   "kernel": main_run["kernel"],
                   "kernel_avg_ms": round(main_run["kernel_avg_ms"], 5),
                   "nodes_per_launch": main_run["nodes_per_launch"],
                   "steps_per_launch": main_run["steps_per_launch"],
                   "bytes_per_node": main_run["bytes_per_node"]},
        "roofline": main_run["roofline"],
        "variants": variants,
        "finite": main_run["finite"],
    }
    if not args.no_copy_ref:
        gbs, ms = copy_ceiling(torch, 9 * w.nx * w.ny * 4)
        line["copy_reference"] = {"GBs": round(gbs, 1), "ms": round(ms, 5), "bytes_each_way": 9 * w.nx * w.ny * 4,
                                  "bulk_frac_of_copy": round(main_run["roofline"]["achieved"] / gbs, 4)}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(W, w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
