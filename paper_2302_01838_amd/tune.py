"""Launch-shape autotuner for the training step.

Times ``vmap_train_step`` on a synthetic workload over a grid of launch shapes and records the
fastest per (GPU arch, hidden width, samples per ray, precision) in ``tune_cache.json`` next to
this file; ``ObjectSet`` reads the cache when it is created without an explicit shape.

Shapes: rays per tile of the hidden-32 tile kernel (fixed when an object stack is created) with
waves per workgroup, or, for workloads with wider models, rays per tile of the cooperative kernel
(``rays_per_tile_wide``, whole rounds of four sub-tiles). Each shape is timed the way the
benchmark times a step: pre-generated batches resident on the device, plain launches, HIP events
around every step; the figure is the median per-step time over ``steps`` steps after a warmup,
and the median of ``repeats`` such runs (each in a fresh object stack).

    python -m paper_2302_01838_amd.tune --workload k50_uneven --precision bf16
    python -m paper_2302_01838_amd.tune --workload stress_k256 --precision bf16
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
from typing import Dict, Iterable, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache.json")


def _key(arch: str, hidden: int, S: int, precision: str) -> str:
    return f"{arch}/H{hidden}/S{S}/{precision}"


def _arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def load_cache(path: str = CACHE) -> Dict[str, dict]:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(hidden: int, S: int, precision: str, arch: Optional[str] = None,
           path: str = CACHE) -> Optional[dict]:
    """Best known launch shape for this model width and batch shape, or None."""
    cache = load_cache(path)
    if arch is None:
        arch = _arch()
    return cache.get(_key(arch, hidden, S, precision))


def _time_shape(scene, dev_batches, precision, rpt, rpt_wide, waves, steps, warmup, log):
    """Median per-step HIP-event time (ms) of one fresh object stack with this shape."""
    import torch
    from . import ObjectSet
    nrays = max(db.n_rays for db in dev_batches)
    objs = ObjectSet(max_objects=scene.n_objects, B=scene.B, hidden=scene.objects[0].hidden,
                     max_hidden=max(o.hidden for o in scene.objects), precision=precision,
                     max_rays=nrays, max_samples_per_ray=scene.S, rays_per_tile=rpt,
                     rays_per_tile_wide=rpt_wide, autotune=False)
    for ob in scene.objects:
        objs.add(ob.norm_centre, ob.norm_scale, hidden=ob.hidden, seed=ob.seed)
    objs.set_launch(waves, 0)
    for i in range(warmup):
        objs.step(dev_batches[i % len(dev_batches)])
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        objs.step(dev_batches[(warmup + i) % len(dev_batches)])
        ev[i + 1].record()
    torch.cuda.synchronize()
    objs.close()
    return statistics.median(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))


def tune(workload: str = "k50_uneven", precision: str = "bf16", steps: int = 100,
         repeats: int = 3, rays_per_tile: Iterable[int] = (), waves: Iterable[int] = (),
         rays_per_tile_wide: Iterable[int] = (), n_batches: int = 4, path: str = CACHE,
         log=print) -> dict:
    """Sweep launch shapes on ``workload``; store and return the best."""
    import scenes
    from . import DeviceBatch
    scene = scenes.make_scene(workload)
    s0 = max(o.join_step for o in scene.objects)  # every object has joined
    dev_batches = [DeviceBatch(scenes.make_batch(scene, s0 + s)) for s in range(n_batches)]
    S = scene.S
    rpw = max(1, 64 // S)
    H = max(o.hidden for o in scene.objects)
    if H == 32:  # the hidden-32 tile kernel: rays per tile x waves per workgroup
        rpts = list(rays_per_tile) or sorted({rpw * m for m in (8, 10, 12, 14, 16, 20, 28)})
        ws = list(waves) or ([4, 8] if precision == "bf16" else [1, 2, 4])
        shapes = [(r, 0, w) for r in rpts for w in ws]
    else:  # wider models: rays per cooperative tile, in whole rounds of four sub-tiles
        rnd = 4 * rpw
        cur = lookup(32, S, precision, path=path) or {}
        rpt32 = int(cur.get("rays_per_tile", 0))
        wides = list(rays_per_tile_wide) or [rnd * m for m in (1, 2, 4, 8, 16, 32)]
        shapes = [(rpt32, rw, int(cur.get("waves", 4))) for rw in wides]
    results = []
    for rpt, rw, w in shapes:
        runs = [_time_shape(scene, dev_batches, precision, rpt, rw, w, steps, 10, log)
                for _ in range(repeats)]
        ms = statistics.median(runs)
        results.append(dict(rays_per_tile=rpt, rays_per_tile_wide=rw, waves=w, grid=0,
                            ms_per_step=ms, runs_ms=runs))
        log(f"[tune] {workload} {precision} rays_per_tile={rpt} rays_per_tile_wide={rw} "
            f"waves={w}: median {ms:.4f} ms/step (runs {', '.join(f'{r:.4f}' for r in runs)})")
    best = min(results, key=lambda r: r["ms_per_step"])
    entry = dict(best, workload=workload, steps=steps, repeats=repeats,
                 timing="median of per-step HIP events, median over repeats", swept=results)
    cache = load_cache(path)
    cache[_key(_arch(), H, S, precision)] = entry
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return entry


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="k50_uneven")
    ap.add_argument("--precision", default="bf16")
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--batches", type=int, default=4, help="distinct pre-generated batches")
    ap.add_argument("--rays-per-tile", type=int, nargs="*", default=[])
    ap.add_argument("--waves", type=int, nargs="*", default=[])
    ap.add_argument("--rays-per-tile-wide", type=int, nargs="*", default=[])
    ap.add_argument("--cache", default=CACHE, help="cache file to update")
    args = ap.parse_args()
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    best = tune(args.workload, args.precision, args.steps, args.repeats, args.rays_per_tile,
                args.waves, args.rays_per_tile_wide, args.batches, path=args.cache)
    print(json.dumps({k: v for k, v in best.items() if k != "swept"}), flush=True)


if __name__ == "__main__":
    main()
