"""Seeded synthetic scenes and ray batches for the vectorised per-object training step.

This module is the only code shared by the FP64 oracle and the GPU path. It generates *inputs*
only: object shapes and bounds, camera rays, sorted sample depths along each ray, and the
observed depth, colour and instance mask of every ray. None of the step's own arithmetic
(encoding, MLP, rendering, loss, adjoint, optimiser) lives here.

The scenes stand in for the paper's Replica workload (Sec. 4.1, "Implementation Details":
about 50 objects per scene, 120 rays x 10 points per object and step, background with 1,200
rays). Replica itself is not used and nothing of its content is reproduced: every scene is made
of analytic spheres and axis-aligned boxes drawn from a seeded generator.

Geometry readings (the paper gives none of this; it trains on real RGB-D frames):

* Each object k has a padded axis-aligned bound (10 % padding on every half-extent). Its
  normalisation centre c_k is the bound's centre and its scale s_k is the largest padded
  half-extent, so the bound maps into [-1, 1]^3 (object-level positional encoding,
  supplement Sec. B).
* Rays are drawn so that each one crosses the object's padded bound, which stands in for the
  paper's sampling of pixels inside the object's 2-D bounding box (Sec. 3.3, "Training
  Objective"). t_n and t_f are the ray's entry and exit of the padded bound.
* The mask M is 1 when the ray's first surface hit is the object itself. D is the range to that
  hit (unit directions, so range and ray parameter coincide) and C is the object's colour. When
  the ray misses, M = 0, D = t_f and C = 0. In rooms, a ray that hits another object first gets
  M = 0 and terminates at that surface (supplement Sec. B, depth-guided sampling).
* Samples along a ray follow the depth-guided scheme of Sec. 3.3 (Eqs. 1 and 2): N_c
  stratified samples in [t_n, t_s] plus N_s samples around t_s, with t_s the observed depth
  when M = 1 and t_f (or the occluder's depth) otherwise. The per-ray list is sorted ascending.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

__all__ = ["WORKLOADS", "SceneObject", "Scene", "make_scene", "make_batch", "make_points",
           "make_encoding_matrix", "batch_samples"]

N_FEATURES = 16          # Gaussian Fourier features per sine/cosine half
ENCODING_SIGMA = 5.0     # B ~ N(0, 25): variance 25, standard deviation 5
BOUND_PADDING = 0.10

# Purpose tags for independent seeded streams.
_SCENE, _B, _RAYS, _NOISE, _POINTS = 1, 2, 3, 4, 5

WORKLOADS: Dict[str, dict] = {
    # K = 4 spheres, 120 rays x 10 samples (5 stratified + 5 ~ N(t_s, 3 cm)), hidden 32.
    "tiny_k4": dict(n_objects=4, shapes="sphere", size=("radius", 0.1, 0.5), box=2.0,
                    rays=("fixed", 120), S=10, n_strat=5, near=("normal", 0.03),
                    depth_noise=0.0, hidden=32, room=None, background=None, waves=None),
    # K = 50 spheres and boxes, rays per object uniform in [60, 600], 20 samples per ray
    # (10 stratified + 10 uniform within +-5 cm of t_s), depth noise 1 cm, hidden 32.
    "k50_uneven": dict(n_objects=50, shapes="mixed", size=("extent", 0.1, 0.8), box=2.0,
                       rays=("uniform", 60, 600), S=20, n_strat=10, near=("uniform", 0.05),
                       depth_noise=0.01, hidden=32, room=None, background=None, waves=None),
    # K = 50 objects in a 6 x 6 x 3 m room plus a hidden-128 background model with 1,200 rays;
    # rays per object lognormal(5, 1) clipped to [16, 4096].
    "room50_background": dict(n_objects=50, shapes="mixed", size=("extent", 0.1, 0.8),
                              box=None, rays=("lognormal", 5.0, 1.0, 16, 4096), S=20,
                              n_strat=10, near=("uniform", 0.05), depth_noise=0.01,
                              hidden=32, room=(6.0, 6.0, 3.0),
                              background=dict(hidden=128, rays=1200), waves=None),
    # K = 256 objects of hidden 64 in a 10 x 10 x 3 m room, rays uniform in [256, 4096],
    # 32 samples per ray (16 + 16); objects join in 8 waves of 32.
    "stress_k256": dict(n_objects=256, shapes="mixed", size=("extent", 0.1, 0.8), box=None,
                        rays=("uniform", 256, 4096), S=32, n_strat=16, near=("uniform", 0.05),
                        depth_noise=0.01, hidden=64, room=(10.0, 10.0, 3.0), background=None,
                        waves=dict(n_waves=8, total_steps=300)),
}


@dataclasses.dataclass
class SceneObject:
    kind: str                 # "sphere", "box" or "room" (the background)
    centre: np.ndarray        # (3,) shape centre, metres
    half: np.ndarray          # (3,) half-extents (sphere: radius repeated)
    rgb: np.ndarray           # (3,) constant colour in [0, 1]
    hidden: int               # MLP width of this object's model
    n_rays: int               # rays per training step
    join_step: int = 0        # first step at which the object has rays
    seed: int = 0             # initialisation seed of the object's model

    @property
    def bound_lo(self) -> np.ndarray:
        pad = 0.0 if self.kind == "room" else BOUND_PADDING
        return self.centre - self.half * (1.0 + pad)

    @property
    def bound_hi(self) -> np.ndarray:
        pad = 0.0 if self.kind == "room" else BOUND_PADDING
        return self.centre + self.half * (1.0 + pad)

    @property
    def norm_centre(self) -> np.ndarray:
        return 0.5 * (self.bound_lo + self.bound_hi)

    @property
    def norm_scale(self) -> float:
        return float(np.max(0.5 * (self.bound_hi - self.bound_lo)))


@dataclasses.dataclass
class Scene:
    name: str
    seed: int
    objects: List[SceneObject]
    S: int
    n_strat: int
    near: tuple
    depth_noise: float
    room: Optional[np.ndarray]       # (3,) room size with the floor corner at the origin
    B: np.ndarray                    # (3, N_FEATURES) float32 encoding matrix

    @property
    def n_objects(self) -> int:
        return len(self.objects)


def _rng(seed: int, *tags: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed)] + [int(t) for t in tags]))


def make_encoding_matrix(seed: int, n_features: int = N_FEATURES,
                         sigma: float = ENCODING_SIGMA) -> np.ndarray:
    """B in R^{3 x F}, entries N(0, sigma^2), rounded to FP32 (the only form either side sees)."""
    return (_rng(seed, _B).standard_normal((3, n_features)) * sigma).astype(np.float32)


def _object_sizes(rng, shapes: str, size: tuple, n: int):
    kinds = []
    halves = np.zeros((n, 3))
    for k in range(n):
        kind = "sphere" if shapes == "sphere" or (shapes == "mixed" and k % 2 == 0) else "box"
        kinds.append(kind)
        lo, hi = size[1], size[2]
        if size[0] == "radius":
            halves[k] = rng.uniform(lo, hi)
        elif kind == "sphere":
            halves[k] = 0.5 * rng.uniform(lo, hi)
        else:
            halves[k] = 0.5 * rng.uniform(lo, hi, size=3)
    return kinds, halves


def _ray_counts(rng, spec: tuple, n: int) -> np.ndarray:
    if spec[0] == "fixed":
        return np.full(n, spec[1], dtype=np.int64)
    if spec[0] == "uniform":
        return rng.integers(spec[1], spec[2] + 1, size=n)
    if spec[0] == "lognormal":
        x = np.round(rng.lognormal(spec[1], spec[2], size=n))
        return np.clip(x, spec[3], spec[4]).astype(np.int64)
    raise ValueError(spec)


def make_scene(name: str, seed: Optional[int] = None) -> Scene:
    """Build the named workload's scene deterministically from ``seed``."""
    cfg = WORKLOADS[name]
    if seed is None:
        seed = list(WORKLOADS).index(name)
    rng = _rng(seed, _SCENE)
    n = cfg["n_objects"]
    kinds, halves = _object_sizes(rng, cfg["shapes"], cfg["size"], n)
    room = None if cfg["room"] is None else np.asarray(cfg["room"], dtype=np.float64)
    centres = np.zeros((n, 3))
    if room is None:
        centres = rng.uniform(-cfg["box"], cfg["box"], size=(n, 3))
    else:
        placed: List[tuple] = []
        for k in range(n):
            for _ in range(10000):
                h = halves[k] * (1.0 + BOUND_PADDING)
                c = rng.uniform(h + 0.05, room - h - 0.05)
                if all(np.any(np.abs(c - c2) >= h + h2) for c2, h2 in placed):
                    break
            else:
                raise RuntimeError("could not place objects without overlap")
            placed.append((c, h))
            centres[k] = c
    rgbs = rng.uniform(0.0, 1.0, size=(n, 3))
    counts = _ray_counts(rng, cfg["rays"], n)
    join = np.zeros(n, dtype=np.int64)
    if cfg["waves"] is not None:
        w = cfg["waves"]
        per = n // w["n_waves"]
        for k in range(n):
            join[k] = (w["total_steps"] * (k // per)) // w["n_waves"]
    objs = [SceneObject(kind=kinds[k], centre=centres[k], half=halves[k], rgb=rgbs[k],
                        hidden=cfg["hidden"], n_rays=int(counts[k]), join_step=int(join[k]),
                        seed=(int(seed) << 32) | k) for k in range(n)]
    if cfg["background"] is not None:
        bg = cfg["background"]
        objs.append(SceneObject(kind="room", centre=0.5 * room, half=0.5 * room,
                                rgb=rng.uniform(0.0, 1.0, size=3), hidden=bg["hidden"],
                                n_rays=bg["rays"], seed=(int(seed) << 32) | n))
    return Scene(name=name, seed=int(seed), objects=objs, S=cfg["S"], n_strat=cfg["n_strat"],
                 near=cfg["near"], depth_noise=cfg["depth_noise"], room=room,
                 B=make_encoding_matrix(seed))


# ----------------------------------------------------------------------------- ray geometry

def _slab(o, d, lo, hi):
    """Entry and exit parameters of rays (o, d) against the box [lo, hi]."""
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / d
        t0 = (lo - o) * inv
        t1 = (hi - o) * inv
    tmin = np.nanmax(np.minimum(t0, t1), axis=-1)
    tmax = np.nanmin(np.maximum(t0, t1), axis=-1)
    return tmin, tmax


def _hit(obj: SceneObject, o, d):
    """Distance to the first surface hit of each ray on ``obj`` (inf where it misses)."""
    if obj.kind == "sphere":
        oc = o - obj.centre
        b = np.sum(oc * d, axis=-1)
        cc = np.sum(oc * oc, axis=-1) - obj.half[0] ** 2
        disc = b * b - cc
        t = -b - np.sqrt(np.maximum(disc, 0.0))
        return np.where((disc >= 0.0) & (t > 0.0), t, np.inf)
    tmin, tmax = _slab(o, d, obj.centre - obj.half, obj.centre + obj.half)
    return np.where((tmin <= tmax) & (tmin > 0.0), tmin, np.inf)


def _unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _room_origins(rng, scene: Scene, n: int):
    out = np.zeros((n, 3))
    todo = np.arange(n)
    while todo.size:
        p = rng.uniform(0.3, scene.room - 0.3, size=(todo.size, 3))
        ok = np.ones(todo.size, dtype=bool)
        for ob in scene.objects:
            if ob.kind == "room":
                continue
            ok &= ~np.all((p >= ob.bound_lo) & (p <= ob.bound_hi), axis=-1)
        out[todo[ok]] = p[ok]
        todo = todo[~ok]
    return out


def _nearest_other(scene: Scene, skip: int, o, d):
    best = np.full(o.shape[0], np.inf)
    for j, ob in enumerate(scene.objects):
        if j == skip or ob.kind == "room":
            continue
        # cheap reject: rays that miss the object's bound cannot hit it
        tmin, tmax = _slab(o, d, ob.centre - ob.half, ob.centre + ob.half)
        cand = np.nonzero((tmin <= tmax) & (tmax > 0.0))[0]
        if cand.size:
            best[cand] = np.minimum(best[cand], _hit(ob, o[cand], d[cand]))
    return best


def _object_rays(rng, scene: Scene, k: int, n: int):
    ob = scene.objects[k]
    if ob.kind == "room":
        o = _room_origins(rng, scene, n)
        d = _unit(rng, n)
        _, t_wall = _slab(o, d, np.zeros(3), scene.room)
        t_other = _nearest_other(scene, k, o, d)
        t_n = np.full(n, 0.05)
        t_f = t_wall
        mask = t_wall < t_other
        depth = np.where(mask, t_wall, np.minimum(t_other, t_wall))
        return o, d, t_n, t_f, mask, depth, depth.copy()
    if scene.room is None:
        o = ob.centre + 3.0 * _unit(rng, n)
    else:
        o = _room_origins(rng, scene, n)
    p = rng.uniform(ob.bound_lo, ob.bound_hi, size=(n, 3))
    d = p - o
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    t_in, t_out = _slab(o, d, ob.bound_lo, ob.bound_hi)
    t_n = np.maximum(t_in, 0.0)
    t_f = t_out
    t_self = _hit(ob, o, d)
    mask = np.isfinite(t_self)
    depth = np.where(mask, t_self, t_f)
    t_s = depth.copy()
    if scene.room is not None:
        t_other = _nearest_other(scene, k, o, d)
        occluded = t_other < np.where(mask, t_self, t_f)
        mask &= ~occluded
        depth = np.where(occluded, t_other, depth)
        t_s = np.where(occluded, np.maximum(t_other, t_n), t_s)
    return o, d, t_n, t_f, mask, depth, t_s


def _samples(rng, scene: Scene, t_n, t_s):
    n = t_n.shape[0]
    nc = scene.n_strat
    ns = scene.S - nc
    u = rng.uniform(0.0, 1.0, size=(n, nc))
    i = np.arange(nc)
    strat = t_n[:, None] + (i[None, :] + u) / nc * (t_s - t_n)[:, None]
    if scene.near[0] == "normal":
        near = t_s[:, None] + scene.near[1] * rng.standard_normal((n, ns))
    else:
        near = t_s[:, None] + rng.uniform(-scene.near[1], scene.near[1], size=(n, ns))
    # samples behind the camera carry no meaning for a depth sensor: clamp them to the origin
    return np.sort(np.maximum(np.concatenate([strat, near], axis=1), 0.0), axis=1)


def make_batch(scene: Scene, step: int = 0, object_ids: Optional[List[int]] = None,
               n_rays: Optional[Dict[int, int]] = None,
               pixel_radius: Optional[float] = None) -> Dict[str, np.ndarray]:
    """One training batch: CSR-segmented rays of the listed objects, as FP32/int32 arrays.

    ``object_ids`` defaults to every object whose ``join_step <= step``. ``n_rays`` overrides
    per-object ray counts (zero allowed). Keys: object_ids [n], ray_offsets [n+1], rays_o
    [R,3], rays_d [R,3], t [R,S], depth [R], rgb [R,3], mask [R], S; with ``pixel_radius``
    (radians) also var [R,S] = (pixel_radius t)^2, the variance of an isotropic Gaussian as wide
    as the pixel's footprint at each sample. Also t_near, t_far [R] (the sampling interval) and
    t_guide [R] (the depth the samples of ``t`` were guided by: the noisy depth where the ray
    hits, else the far bound or the occluder), for sampling on the device.
    """
    if object_ids is None:
        object_ids = [k for k, ob in enumerate(scene.objects) if ob.join_step <= step]
    counts = [int(scene.objects[k].n_rays if n_rays is None or k not in n_rays else n_rays[k])
              for k in object_ids]
    parts = []
    for k, n in zip(object_ids, counts):
        rng = _rng(scene.seed, _RAYS, step, k)
        o, d, t_n, t_f, mask, depth, t_s = _object_rays(rng, scene, k, n)
        if scene.depth_noise > 0.0:
            nrng = _rng(scene.seed, _NOISE, step, k)
            noisy = depth + scene.depth_noise * nrng.standard_normal(n)
            depth = np.where(mask, noisy, depth)
            t_s = np.where(mask, depth, t_s)
        t = _samples(rng, scene, t_n, t_s)
        rgb = np.where(mask[:, None], scene.objects[k].rgb[None, :], 0.0)
        parts.append((o, d, t, depth, rgb, mask.astype(np.float64), t_n, t_f, t_s))
    S = scene.S
    offs = np.zeros(len(object_ids) + 1, dtype=np.int32)
    offs[1:] = np.cumsum(counts)

    def cat(i, shape):
        arrs = [p[i] for p in parts if p[i].shape[0]]
        return (np.concatenate(arrs, axis=0) if arrs else np.zeros(shape)).astype(np.float32)

    t = cat(2, (0, S))
    # FP32 rounding can break the order of nearly equal samples; the step requires sorted t.
    t = np.sort(t, axis=1)
    out = dict(object_ids=np.asarray(object_ids, dtype=np.int32), ray_offsets=offs,
               rays_o=cat(0, (0, 3)), rays_d=cat(1, (0, 3)), t=t, depth=cat(3, (0,)),
               rgb=cat(4, (0, 3)), mask=cat(5, (0,)), S=S,
               t_near=cat(6, (0,)), t_far=cat(7, (0,)), t_guide=cat(8, (0,)))
    if pixel_radius is not None:
        out["var"] = (np.float64(pixel_radius) * t.astype(np.float64)) ** 2
        out["var"] = out["var"].astype(np.float32)
    return out


def batch_samples(batch) -> int:
    return int(batch["t"].shape[0] * batch["S"])


def make_points(scene: Scene, k: int, n: int, seed: int = 0) -> np.ndarray:
    """n world-frame query points, uniform in object k's padded bound, FP32 [n, 3]."""
    ob = scene.objects[k]
    rng = _rng(scene.seed, _POINTS, seed, k)
    return rng.uniform(ob.bound_lo, ob.bound_hi, size=(n, 3)).astype(np.float32)
