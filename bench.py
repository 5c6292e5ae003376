#!/usr/bin/env python3
"""Benchmark of the vectorised per-object training step on one MI355X.

Workload: 50 objects (spheres and boxes), rays per object uniform in [60, 600] drawn once, 20
samples per ray (10 stratified + 10 within +-5 cm of the surface), hidden 32, 4 hidden layers,
Adam lr 1e-3. Batches are synthetic, pre-generated and resident in HBM before timing. The same
batches train a fresh model stack twice: the plain FP32 form and the BF16-MFMA form; each form
runs `warmup` untimed steps and then `steps` timed steps.

Prints one JSON line: the BF16 form's ray-samples/s as `value`, both forms' object-steps/s and
ray-samples/s, their final losses (mean total loss over the last 10 steps) and whether they
match within 2e-2, the roofline of the dominant kernel (the fused tile kernel, timed with HIP
events on its launch stream), and the FP64 oracle timed on the host on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "k50_uneven"
WORKLOAD_TEXT = {
    "k50_uneven": "K=50 objects, rays/object U[60,600], 20 samples/ray, hidden 32, 4 hidden "
                  "layers, Adam lr 1e-3",
    "room50_background": "K=50 objects (hidden 32, rays lognormal(5,1) in [16,4096]) + hidden-128 "
                         "background (1,200 rays), 20 samples/ray, 6x6x3 m room, BF16",
    "stress_k256": "K=256 objects, hidden 64, rays/object U[256,4096], 32 samples/ray, "
                   "10x10x3 m room, all objects joined, BF16",
}


def flop_per_sample(H: int) -> int:
    """Algorithmic FLOPs of one training step per sample for width H, four hidden layers, E = 32,
    four outputs: forward 32H + 3H^2 + 4H MACs; backward all weight gradients (the same count)
    plus input gradients of layers 2..5 (3H^2 + 4H); 2 FLOPs per MAC. H = 32: 23,296. No
    recomputation, padding, encoding or rendering work counted."""
    fwd = 32 * H + 3 * H * H + 4 * H
    return 2 * (fwd + fwd + 3 * H * H + 4 * H)


FLOP_PER_SAMPLE_H32 = flop_per_sample(32)
PEAK = {"bf16": 2.5e15, "fp32": 157.3e12}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "tile_kernel_traffic_k50_uneven.md")


def tile_kernel_fingerprint() -> str:
    """SHA-256 of the source that defines the hidden-32 tile kernel: vmap_kernels.hip from the
    activation types to the end of k_step_tiles, plus vmap_internal.h, vmap_math.h and
    vmap_bf16.h."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2302_01838_amd", "csrc")
    k = open(os.path.join(csrc, "vmap_kernels.hip")).read()
    a = k.index("// Activations of one 32-sample pass")
    b = k.index("// Tile kernel for wide models")
    h = hashlib.sha256(k[a:b].encode())
    for name in ("vmap_internal.h", "vmap_math.h", "vmap_bf16.h"):
        h.update(open(os.path.join(csrc, name)).read().encode())
    return h.hexdigest()


def measured_traffic(precision: str, rays_per_tile: int, waves: int, split_step: bool = False):
    """HBM bytes per launch of the timed kernel from the committed counter summary, or None if
    the summary is missing, was taken on a different version of the kernel source, or holds no
    figure for this launch shape and step form."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if line.startswith("- ") and ":" in line:
            key, val = line[2:].split(":", 1)
            fields[key.strip()] = val.strip().strip("`")
    if fields.get("kernel source sha256") != tile_kernel_fingerprint():
        return None
    form = "split" if split_step else "table"
    val = fields.get(f"traffic bytes per launch ({precision}, rays_per_tile {rays_per_tile}, "
                     f"waves {waves}, {form})")
    return int(val.replace(",", "")) if val else None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def first_full_step(scene):
    """First step at which every object of the scene has joined."""
    return max(o.join_step for o in scene.objects)


def gen_batches(scene, n):
    import scenes
    s0 = first_full_step(scene)
    return [scenes.make_batch(scene, s0 + step) for step in range(n)]


def batch_flops(scene, db) -> float:
    """Algorithmic FLOPs of one step over a device batch (per-object widths)."""
    offs = np.asarray(db.ray_offsets)
    ids = np.asarray(db.object_ids)
    return float(sum(flop_per_sample(scene.objects[int(k)].hidden) * int(offs[j + 1] - offs[j]) * db.S
                     for j, k in enumerate(ids)))


def run_form(precision, scene, dev_batches, steps, warmup, graph, timing_steps,
             rays_per_tile_wide=0, split_step=False, device_sampling=False):
    import torch
    import paper_2302_01838_amd as vm
    nrays = max(db.n_rays for db in dev_batches)
    objs = vm.ObjectSet(max_objects=scene.n_objects, B=scene.B, hidden=scene.objects[0].hidden,
                        max_hidden=max(o.hidden for o in scene.objects), precision=precision,
                        max_rays=nrays, max_samples_per_ray=scene.S,
                        rays_per_tile_wide=rays_per_tile_wide, split_step=split_step)
    for ob in scene.objects:
        objs.add(ob.norm_centre, ob.norm_scale, hidden=ob.hidden, seed=ob.seed)
    objs.set_graph_mode(graph)
    # with device sampling each step first draws its batch's sample depths on the GPU (Eqs. 1-2,
    # into the batch's t) from the rays' bounds and guide depths, with a new seed per step
    sigma = scene.near[1] if scene.near[0] == "normal" else scene.near[1] / 3.0 ** 0.5
    draws = [0]

    def step(db, losses=None):
        if device_sampling:
            tn, tf, tg = db.sampling
            objs.sample_rays(tn, tf, tg, db.S, scene.n_strat, sigma, seed=draws[0], out=db["t"])
            draws[0] += 1
        objs.step(db, losses)
    n_obj = scene.n_objects
    loss_hist = torch.zeros(warmup + steps, n_obj, device="cuda")
    for i in range(warmup):
        step(dev_batches[i % len(dev_batches)], loss_hist[i])
    torch.cuda.synchronize()
    # two events only: an event between steps is a marker the GPU waits on (about 5 us each)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for i in range(steps):
        step(dev_batches[(warmup + i) % len(dev_batches)], loss_hist[warmup + i])
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    event_ms_per_step = ev0.elapsed_time(ev1) / steps
    losses = loss_hist.sum(1).cpu().numpy()
    # per-step HIP events in a separate pass (an event between steps costs a few microseconds of
    # idle GPU, so the headline loop above has none): the median over steps 10..end
    n_ev = min(steps, 100) + 10
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n_ev + 1)]
    evs[0].record()
    for i in range(n_ev):
        step(dev_batches[(warmup + i) % len(dev_batches)])
        evs[i + 1].record()
    torch.cuda.synchronize()
    per_step = [evs[i].elapsed_time(evs[i + 1]) for i in range(10, n_ev)]
    event_ms_median = statistics.median(per_step)
    samples = [dev_batches[(warmup + i) % len(dev_batches)].n_samples for i in range(steps)]
    active = [int(np.sum(np.diff(dev_batches[(warmup + i) % len(dev_batches)].ray_offsets) > 0))
              for i in range(steps)]
    # dominant kernel: time the tile kernel with events on its stream (plain launches)
    objs.set_graph_mode(False)
    objs.kernel_timing(1)
    for i in range(timing_steps):
        step(dev_batches[i % len(dev_batches)])
    torch.cuda.synchronize()
    k_ms, k_n = objs.kernel_timing(0)
    k_samples = statistics.mean(dev_batches[i % len(dev_batches)].n_samples for i in range(timing_steps))
    k_flops = statistics.mean(batch_flops(scene, dev_batches[i % len(dev_batches)])
                              for i in range(timing_steps))
    scale, skipped, err = objs.step_info()
    launch = {"tuned": bool(objs.tuned), "rays_per_tile": objs.rays_per_tile,
              "waves": objs.waves, "grid": objs.grid, "split_step": bool(split_step)}
    objs.close()
    return dict(
        precision=precision,
        wall_s=wall,
        ms_per_step=1e3 * wall / steps,
        event_ms_per_step=event_ms_per_step,
        event_ms_per_step_median=event_ms_median,
        ray_samples_per_s=sum(samples) / wall,
        object_steps_per_s=sum(active) / wall,
        final_loss=float(np.mean(losses[-10:])),
        first_loss=float(losses[0]),
        loss_scale=scale,
        skipped_last=skipped,
        device_error=err,
        kernel_ms=k_ms,
        kernel_launches=k_n,
        kernel_samples=k_samples,
        kernel_flops=k_flops,
        launch=launch,
    )


def sweep_hidden(widths, steps, n_objects=50, graph=False):
    """Vectorised vs sequential training step over hidden widths (Sec. 4.3, Fig. "ablative
    vectorised", right): n_objects objects of one width, 120 rays x 10 samples each, BF16. Widths
    32, 64 and 128 run the fused tile kernels, 16 the width-32 one zero-padded, 256 and up the
    layered path. Returns ms per step."""
    import dataclasses
    import torch
    import scenes
    import paper_2302_01838_amd as vm
    base = scenes.make_scene("tiny_k4")
    out = []
    for H in widths:
        rng = np.random.default_rng(H)
        objs_ = []
        for k in range(n_objects):
            o = base.objects[k % base.n_objects]
            objs_.append(dataclasses.replace(o, centre=rng.uniform(-2, 2, size=3), hidden=H,
                                             seed=(1 << 41) + k))
        sc = dataclasses.replace(base, objects=objs_)
        batches = [scenes.make_batch(sc, i) for i in range(3)]
        full = [vm.DeviceBatch(b) for b in batches]
        per_obj = []
        for b in batches:
            offs = b["ray_offsets"]
            row = []
            for j in range(n_objects):
                sl = slice(offs[j], offs[j + 1])
                sub = {f: b[f][sl] for f in ("rays_o", "rays_d", "t", "depth", "rgb", "mask")}
                sub["object_ids"] = b["object_ids"][j:j + 1]
                sub["ray_offsets"] = np.array([0, offs[j + 1] - offs[j]], dtype=np.int32)
                sub["S"] = b["S"]
                row.append(vm.DeviceBatch(sub))
            per_obj.append(row)
        res = {"hidden": H, "path": ("fused tile kernel" if H in (32, 64, 128) else
                                     "fused tile kernel, zero-padded to 32" if H == 16 else "layered")}
        for mode in ("vectorised", "sequential"):
            objs = vm.ObjectSet(max_objects=n_objects, B=sc.B, hidden=H, precision="bf16",
                                max_rays=full[0].n_rays, max_samples_per_ray=sc.S)
            for ob in sc.objects:
                objs.add(ob.norm_centre, ob.norm_scale, hidden=H, seed=ob.seed)
            res["params_per_object"] = objs.n_params[0]
            objs.set_graph_mode(graph)

            def one(i):
                if mode == "vectorised":
                    objs.step(full[i % 3])
                else:
                    for db in per_obj[i % 3]:
                        objs.step(db)
            for i in range(3):
                one(i)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(steps):
                one(i)
            torch.cuda.synchronize()
            res[mode + "_ms"] = 1e3 * (time.perf_counter() - t0) / steps
            objs.close()
        log(f"sweep H={H}: vectorised {res['vectorised_ms']:.3f} ms, "
            f"sequential {res['sequential_ms']:.3f} ms")
        out.append(res)
    return out


def sweep_objects(counts, steps, precision, graph):
    """Vectorised vs sequential training step over object counts (the paper's Sec. 4.3 ablation,
    on synthetic scenes shaped like its workload: 120 rays x 10 samples per object, hidden 32).

    Vectorised: one vmap_train_step over all objects. Sequential: one vmap_train_step per object
    (a per-object loop of the same kernels). Returns ms per step for each count.
    """
    import dataclasses
    import torch
    import scenes
    import paper_2302_01838_amd as vm
    base = scenes.make_scene("tiny_k4")
    out = []
    for K in counts:
        rng = np.random.default_rng(K)
        objs_ = []
        for k in range(K):
            o = base.objects[k % base.n_objects]
            objs_.append(dataclasses.replace(o, centre=rng.uniform(-2, 2, size=3),
                                             seed=(1 << 40) + k))
        sc = dataclasses.replace(base, objects=objs_)
        batches = [scenes.make_batch(sc, i) for i in range(3)]
        full = [vm.DeviceBatch(b) for b in batches]
        per_obj = []
        for b in batches:
            offs = b["ray_offsets"]
            row = []
            for j in range(K):
                sl = slice(offs[j], offs[j + 1])
                sub = {f: b[f][sl] for f in ("rays_o", "rays_d", "t", "depth", "rgb", "mask")}
                sub["object_ids"] = b["object_ids"][j:j + 1]
                sub["ray_offsets"] = np.array([0, offs[j + 1] - offs[j]], dtype=np.int32)
                sub["S"] = b["S"]
                row.append(vm.DeviceBatch(sub))
            per_obj.append(row)
        res = {"objects": K}
        for mode in ("vectorised", "sequential"):
            objs = vm.ObjectSet(max_objects=K, B=sc.B, hidden=32, precision=precision,
                                max_rays=full[0].n_rays, max_samples_per_ray=sc.S)
            for ob in sc.objects:
                objs.add(ob.norm_centre, ob.norm_scale, hidden=32, seed=ob.seed)
            objs.set_graph_mode(graph)

            def one(i):
                if mode == "vectorised":
                    objs.step(full[i % 3])
                else:
                    for db in per_obj[i % 3]:
                        objs.step(db)
            for i in range(3):
                one(i)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(steps):
                one(i)
            torch.cuda.synchronize()
            res[mode + "_ms"] = 1e3 * (time.perf_counter() - t0) / steps
            objs.close()
        log(f"sweep K={K}: vectorised {res['vectorised_ms']:.3f} ms, "
            f"sequential {res['sequential_ms']:.3f} ms")
        out.append(res)
    return out


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def host_cores(cap: int = 16) -> int:
    """Cores this process may use, at most ``cap`` (a one-GPU machine's share of its host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


# The oracle legs read the scene and batches from here (worker processes inherit them by fork).
_ORACLE_INPUT = {}


def _oracle_run(objects, budget_s):
    """The FP64 oracle, one BLAS thread, on the given objects' steps in order (object k's step n
    is its rays of batch n) until ``budget_s`` seconds have passed. Returns (samples, object
    steps, seconds)."""
    import oracle
    from threadpoolctl import threadpool_limits
    scene, batches = _ORACLE_INPUT["scene"], _ORACLE_INPUT["batches"]
    mine = set(objects)
    states = {k: oracle.ObjectState(oracle.xavier_init(o.seed, o.hidden, 4, 32), o.hidden, 4,
                                    o.norm_centre, o.norm_scale)
              for k, o in enumerate(scene.objects) if k in mine}
    samples = obj_steps = 0
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        for b in batches:
            offs = b["ray_offsets"]
            for j, k in enumerate(b["object_ids"]):
                if int(k) not in mine:
                    continue
                sl = slice(offs[j], offs[j + 1])
                sub = {f: b[f][sl] for f in ("rays_o", "rays_d", "t", "depth", "rgb", "mask")}
                sub["object_ids"] = b["object_ids"][j:j + 1]
                sub["ray_offsets"] = np.array([0, offs[j + 1] - offs[j]], dtype=np.int32)
                sub["S"] = b["S"]
                oracle.step(states, sub, scene.B)
                samples += sub["t"].size
                obj_steps += int(offs[j + 1] > offs[j])
                if time.perf_counter() - t0 > budget_s:
                    return samples, obj_steps, time.perf_counter() - t0
    return samples, obj_steps, time.perf_counter() - t0


def _oracle_worker(args):
    return _oracle_run(*args)


def cpu_baseline(scene, batches, budget_s=15.0, workload=WORKLOAD):
    """The FP64 oracle on the host in two legs of about budget_s / 2 seconds each: one thread
    (objects one after another), and all cores (objects dealt to one worker process per core,
    each with one BLAS thread, each running its objects' steps in order). Must run before the
    GPU is initialised: the worker processes are forked."""
    import multiprocessing as mp
    _ORACLE_INPUT.update(scene=scene, batches=batches)
    leg = budget_s / 2.0
    all_ids = list(range(scene.n_objects))
    s1, o1, t1 = _oracle_run(all_ids, leg)
    P = min(host_cores(), scene.n_objects)
    parts = [(all_ids[w::P], leg) for w in range(P)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(P) as pool:
        res = pool.map(_oracle_worker, parts)
    wall = time.perf_counter() - t0
    sP, oP = sum(r[0] for r in res), sum(r[1] for r in res)
    sample = (f"the {workload} workload's batches from the initial models, each object's steps in "
              f"order; all cores: {oP} object-steps ({sP} samples) in {wall:.1f} s over {P} "
              f"worker processes of one BLAS thread; one thread: {o1} object-steps ({s1} samples) "
              f"in {t1:.1f} s; FP64 numpy")
    return dict(value=sP / wall, unit="ray-samples/s", cores=P, kind="oracle", sample=sample,
                object_steps_per_s=oP / wall, seconds=wall, cpu_model=cpu_model(),
                one_thread={"value": s1 / t1, "unit": "ray-samples/s", "cores": 1,
                            "object_steps_per_s": o1 / t1, "seconds": t1})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--graph", type=int, default=0,
                    help="replay the step as a hipGraph (slower here: hipGraphLaunch costs more "
                         "host time than the three plain launches)")
    ap.add_argument("--split-step", action="store_true",
                    help="a separate work-list launch before the tile kernel (default: the tile "
                         "kernel builds its work list)")
    ap.add_argument("--distinct-batches", type=int, default=0,
                    help="distinct pre-generated batches (default: warmup + steps)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--forms", default=None,
                    help="comma-separated precisions (default fp32,bf16; bf16 with hidden 128)")
    ap.add_argument("--rays-per-tile-wide", type=int, default=0,
                    help="tile size of objects wider than 32 (0: the library default)")
    ap.add_argument("--workload", default=WORKLOAD, choices=sorted(WORKLOAD_TEXT),
                    help="k50_uneven is the headline workload; the others are reported in the docs")
    ap.add_argument("--device-sampling", action="store_true",
                    help="draw every step's sample depths on the GPU (vmap_sample_rays) before "
                         "the step: the end-to-end rate; not the headline configuration")
    ap.add_argument("--hidden", type=int, default=0,
                    help="give every object of the workload this width (the layered widths 16, "
                         "256, 512, 1024 train in BF16 only); not the headline configuration")
    ap.add_argument("--sweep-objects", type=int, nargs="*", default=None,
                    help="only run the vectorised-vs-sequential sweep over these object counts")
    ap.add_argument("--sweep-hidden", type=int, nargs="*", default=None,
                    help="only run the vectorised-vs-sequential sweep over these hidden widths "
                         "(BF16, 50 objects of 120 rays x 10 samples)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run 5 device-to-device copies of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy_mib:
        import torch
        n = args.calibrate_copy_mib * (1 << 20) // 4
        x = torch.ones(n, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": n * 4, "launches": 5}), flush=True)
        return
    if args.forms is None:
        args.forms = "bf16" if (args.workload != WORKLOAD or args.hidden) else "fp32,bf16"
    if args.sweep_hidden is not None:
        widths = args.sweep_hidden or [16, 32, 64, 128, 256, 512, 1024]
        res = sweep_hidden(widths, max(1, min(args.steps, 20)), graph=bool(args.graph))
        print(json.dumps({"sweep": "vectorised_vs_sequential_hidden", "precision": "bf16",
                          "objects": 50, "rays_per_object": 120, "samples_per_ray": 10,
                          "results": res}), flush=True)
        return
    if args.sweep_objects is not None:
        counts = args.sweep_objects or [1, 10, 20, 30, 40, 50, 100, 150, 200]
        res = sweep_objects(counts, max(1, min(args.steps, 50)), args.forms.split(",")[-1],
                            bool(args.graph))
        print(json.dumps({"sweep": "vectorised_vs_sequential", "precision": args.forms.split(",")[-1],
                          "rays_per_object": 120, "samples_per_ray": 10, "hidden": 32,
                          "results": res}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the step has no "
              "cross-GPU exchange; objects would be sharded across GPUs by object)",
              file=sys.stderr)
        sys.exit(2)

    import scenes

    scene = scenes.make_scene(args.workload)
    if args.hidden:
        import dataclasses
        scene = dataclasses.replace(scene, objects=[dataclasses.replace(o, hidden=args.hidden)
                                                    for o in scene.objects])
    headline = args.workload == WORKLOAD and not args.hidden and not args.device_sampling
    n_batches = args.distinct_batches or (args.warmup + args.steps)
    log(f"generating {n_batches} batches of {args.workload}")
    batches = gen_batches(scene, n_batches)
    # the oracle first, before anything touches the GPU (its all-cores leg forks workers);
    # --cpu-budget 0 skips it (profiled runs: a profiler initialises the GPU before the program)
    cpu = None
    if args.cpu_budget > 0:
        log(f"cpu baseline: oracle for about {args.cpu_budget:.0f} s (one thread, then all cores)")
        cpu = cpu_baseline(scene, batches, args.cpu_budget, args.workload)

    import torch
    import paper_2302_01838_amd as vm

    vm.load_library()
    dev_batches = [vm.DeviceBatch(b) for b in batches]
    if args.device_sampling:  # each batch's ray bounds and guide depths, resident like the batch
        for db, b in zip(dev_batches, batches):
            db.sampling = tuple(torch.as_tensor(b[k]).to("cuda").contiguous()
                                for k in ("t_near", "t_far", "t_guide"))
    torch.cuda.synchronize()

    forms = {}
    for prec in args.forms.split(","):
        log(f"form {prec}: {args.warmup} warmup + {args.steps} timed steps")
        forms[prec] = run_form(prec, scene, dev_batches, args.steps, args.warmup,
                               bool(args.graph), timing_steps=min(args.steps, 50),
                               rays_per_tile_wide=args.rays_per_tile_wide,
                               split_step=args.split_step, device_sampling=args.device_sampling)
        log(f"form {prec}: {forms[prec]['ms_per_step']:.4f} ms/step, "
            f"{forms[prec]['ray_samples_per_s']:.4g} samples/s, final loss "
            f"{forms[prec]['final_loss']:.6g}")

    head = forms.get("bf16") or next(iter(forms.values()))
    prec = head["precision"]
    matched = None
    if "bf16" in forms and "fp32" in forms:
        matched = abs(forms["bf16"]["final_loss"] - forms["fp32"]["final_loss"]) <= \
            2e-2 * abs(forms["fp32"]["final_loss"])
    flops = head["kernel_flops"]
    achieved = flops / (head["kernel_ms"] * 1e-3) if head["kernel_ms"] > 0 else 0.0
    shape = head.get("launch", {})
    traffic = (measured_traffic(prec, shape.get("rays_per_tile", 0), shape.get("waves", 0),
                                shape.get("split_step", False))
               if headline else None)
    if not headline:
        kname = ("tile kernels of the step (cooperative kernel of the wide models, with the "
                 "hidden-32 tile kernel where present), events around all of a step's tile launches")
    elif shape.get("split_step"):
        kname = "tile kernel (encode+MLP+render+loss+backward; work list launched apart)"
    else:
        kname = "tile kernel (work list built in-kernel, encode+MLP+render+loss+backward)"
    roofline = dict(bound="mfma", achieved=achieved / 1e12, peak=PEAK[prec] / 1e12, unit="TFLOP/s",
                    frac=achieved / PEAK[prec], traffic=traffic,
                    kernel=kname,
                    kernel_avg_ms=head["kernel_ms"], flop_per_launch=flops)
    out = {
        "metric": "object-steps/s and ray-samples/s at K=50, BF16 vs FP32, at matched final loss",
        "value": head["ray_samples_per_s"],
        "unit": "ray-samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload]
                   + (f", every object at hidden {args.hidden}" if args.hidden else "")
                   + (", sample depths drawn on the GPU every step" if args.device_sampling else ""),
                   "objects": scene.n_objects, "samples_per_step": dev_batches[0].n_samples,
                   "graph": bool(args.graph), "parallelism": "single GPU",
                   "launch": {k: v for k, v in head.get("launch", {}).items()}},
        "object_steps_per_s": head["object_steps_per_s"],
        "forms": {k: {kk: v[kk] for kk in ("ray_samples_per_s", "object_steps_per_s", "ms_per_step",
                                           "event_ms_per_step", "event_ms_per_step_median",
                                           "final_loss", "first_loss",
                                           "loss_scale", "skipped_last", "device_error",
                                           "kernel_ms")} for k, v in forms.items()},
        "matched_final_loss": matched,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "host": {"cpu": cpu_model(), "nproc": os.cpu_count(), "cores_used": host_cores()},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
