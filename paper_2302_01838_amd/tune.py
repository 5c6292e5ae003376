"""Launch-shape autotuner for the training step.

Times ``vmap_train_step`` on a synthetic workload over a grid of launch shapes — rays per tile
(fixed when an object stack is created), waves per workgroup and grid size (0 = one workgroup per
tile, otherwise a persistent grid) — and records the fastest per (GPU arch, hidden width, samples
per ray, precision) in ``tune_cache.json`` next to this file. ``ObjectSet`` reads the cache when
it is created without an explicit ``rays_per_tile``.

    python -m paper_2302_01838_amd.tune --workload k50_uneven --precision bf16
"""
from __future__ import annotations

import argparse
import json
import os
import time
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
    """Best known launch shape for this model and batch shape, or None."""
    cache = load_cache(path)
    if arch is None:
        arch = _arch()
    return cache.get(_key(arch, hidden, S, precision))


def _time_shape(scene, dev_batches, precision, rpt, waves, grid, steps, graph):
    import torch
    from . import ObjectSet
    nrays = max(db.n_rays for db in dev_batches)
    objs = ObjectSet(max_objects=scene.n_objects, B=scene.B, hidden=scene.objects[0].hidden,
                     max_hidden=max(o.hidden for o in scene.objects), precision=precision,
                     max_rays=nrays, max_samples_per_ray=scene.S, rays_per_tile=rpt,
                     autotune=False)
    for ob in scene.objects:
        objs.add(ob.norm_centre, ob.norm_scale, hidden=ob.hidden, seed=ob.seed)
    objs.set_launch(waves, grid)
    objs.set_graph_mode(graph)
    for i in range(3):
        objs.step(dev_batches[i % len(dev_batches)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        objs.step(dev_batches[i % len(dev_batches)])
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    objs.close()
    return dt


def tune(workload: str = "k50_uneven", precision: str = "bf16", steps: int = 20,
         rays_per_tile: Iterable[int] = (), waves: Iterable[int] = (2, 4),
         grids: Iterable[int] = (0,), graph: bool = False, path: str = CACHE,
         log=print) -> dict:
    """Sweep launch shapes on ``workload``; store and return the best."""
    import scenes
    from . import DeviceBatch
    scene = scenes.make_scene(workload)
    dev_batches = [DeviceBatch(scenes.make_batch(scene, s)) for s in range(4)]
    S = scene.S
    rpw = max(1, 64 // S)
    rpts = list(rays_per_tile) or sorted({rpw * m for m in (2, 4, 6, 8, 10, 12, 16, 20)})
    results = []
    for rpt in rpts:
        for w in waves:
            for g in grids:
                dt = _time_shape(scene, dev_batches, precision, rpt, w, g, steps, graph)
                results.append(dict(rays_per_tile=rpt, waves=w, grid=g, ms_per_step=dt * 1e3))
                log(f"[tune] {workload} {precision} rays_per_tile={rpt} waves={w} grid={g}: "
                    f"{dt * 1e3:.4f} ms/step")
    best = min(results, key=lambda r: r["ms_per_step"])
    hidden = scene.objects[0].hidden
    entry = dict(best, workload=workload, swept=results)
    cache = load_cache(path)
    cache[_key(_arch(), hidden, S, precision)] = entry
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return entry


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="k50_uneven")
    ap.add_argument("--precision", default="bf16")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--rays-per-tile", type=int, nargs="*", default=[])
    ap.add_argument("--waves", type=int, nargs="*", default=[2, 4])
    ap.add_argument("--grids", type=int, nargs="*", default=[0])
    ap.add_argument("--graph", type=int, default=0)
    ap.add_argument("--cache", default=CACHE, help="cache file to update")
    args = ap.parse_args()
    import sys
    sys.path.insert(0, os.path.dirname(HERE))
    best = tune(args.workload, args.precision, args.steps, args.rays_per_tile, args.waves,
                args.grids, bool(args.graph), path=args.cache)
    print(json.dumps({k: v for k, v in best.items() if k != "swept"}))


if __name__ == "__main__":
    main()
