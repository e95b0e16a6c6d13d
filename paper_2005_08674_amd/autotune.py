"""Launch-shape autotuner with a JSON cache.

The library times every compiled launch shape on a live lattice (median of
repeated launches): ``lbm_autotune`` the single-step launch (the fused edge +
bulk kernel), ``lbm_autotune_two_step`` the multi-step sweeps (two or three
steps per launch) where the lattice supports them.  The fastest per step wins.  This module keeps the winners in
``tuning/tiles.json`` keyed by (GPU architecture, lattice size, storage), so
later runs reuse a measured choice instead of re-timing, and records every
candidate's time.

    python -m paper_2005_08674_amd.autotune --size 4096 --stores f32,f16,bf16,f64 --reps 15
"""
from __future__ import annotations

import argparse
import json
import os
import time

from . import lbm as L

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "tiles.json")


def arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def key(nx: int, ny: int, store: str, gpu_arch: str | None = None) -> str:
    return f"{gpu_arch or arch()}:{nx}x{ny}:{store}"


def load_cache(path: str = CACHE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(nx: int, ny: int, store: str, path: str = CACHE, gpu_arch: str | None = None):
    """Cached (tile name, two-step shape name or None) for this lattice, or None."""
    entry = load_cache(path).get(key(nx, ny, store, gpu_arch))
    if not entry:
        return None
    names = [L.lbm_tile_describe(i) for i in range(L.lbm_tile_count())]
    twos = [L.lbm_two_step_describe(i) for i in range(L.lbm_two_step_count())]
    two = entry.get("two_step")
    if entry["tile"] not in names or (two is not None and two not in twos):
        return None
    return entry["tile"], two


def apply(lattice, store: str, path: str = CACHE) -> str | None:
    """Set the cached choice on a Lattice; returns its description, or None if not cached."""
    hit = lookup(lattice.nx, lattice.ny, store, path)
    if hit is None:
        return None
    tile, two = hit
    names = [L.lbm_tile_describe(i) for i in range(L.lbm_tile_count())]
    L.lbm_set_tile(lattice.ctx, names.index(tile))
    if two is not None:
        twos = [L.lbm_two_step_describe(i) for i in range(L.lbm_two_step_count())]
        L.lbm_set_two_step(lattice.ctx, twos.index(two))
    else:
        L.lbm_set_two_step(lattice.ctx, -1)
    return tile if two is None else f"{tile} | {two}"


def tune(lattice, store: str, reps: int = 10, path: str | None = CACHE) -> dict:
    """Time every candidate on ``lattice``: single-step tiles, then the multi-step shapes (two and three
    steps per launch) if the lattice supports them; keep the fastest per step, select it, and record it
    in the cache."""
    best, times = L.lbm_autotune(lattice.ctx, reps)
    names = [L.lbm_tile_describe(i) for i in range(L.lbm_tile_count())]
    entry = {"tile": names[best], "ms": times[best], "reps": reps,
             "candidates": {n: round(t, 5) for n, t in zip(names, times)},
             "two_step": None, "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    try:
        b2, t2 = L.lbm_autotune_two_step(lattice.ctx, reps)
    except L.LbmError:
        b2 = None
    if b2 is not None:
        twos = [L.lbm_two_step_describe(i) for i in range(L.lbm_two_step_count())]
        entry["two_step_candidates"] = {n: round(t, 5) for n, t in zip(twos, t2)}
        if t2[b2] < times[best]:  # both per step (a multi-step launch advances two or three)
            entry["two_step"] = twos[b2]
            entry["two_step_ms"] = t2[b2]
        else:
            L.lbm_set_two_step(lattice.ctx, -1)
    if path:
        cache = load_cache(path)
        cache[key(lattice.nx, lattice.ny, store)] = entry
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return entry


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--size", type=int, default=4096, help="square lattice side (pulse workload)")
    ap.add_argument("--stores", default="f32,f16,bf16,f64")
    ap.add_argument("--reps", type=int, default=15)
    ap.add_argument("--cache", default=CACHE)
    args = ap.parse_args()
    from . import workloads as W
    from .lattice import Lattice
    w = W.pulses_4096(n=args.size)
    for st in args.stores.split(","):
        lat = Lattice(w.nx, w.ny, w.tau, w.fields, store=st)
        lat.step(5)
        e = tune(lat, st, args.reps, args.cache)
        two = f", multi-step {e['two_step']} ({e['two_step_ms']:.4f} ms per step)" if e["two_step"] else ""
        print(f"{key(w.nx, w.ny, st)} -> {e['tile']} ({e['ms']:.4f} ms){two}", flush=True)
        lat.close()


if __name__ == "__main__":
    main()
