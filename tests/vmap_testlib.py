"""Shared helpers of the GPU parity tests: build a library object set and the oracle's twin
from the same seeded scene, and compare results norm-wise."""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle
import scenes

FP32_TOL = 1e-5
BF16_TOL = 2e-2
BF16_VS_BF16_ORACLE = 2e-3


def relerr(x, ref) -> float:
    """Norm-wise relative error ||x - ref|| / ||ref||; exact zeros must match exactly."""
    x = np.asarray(x, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    nr = np.linalg.norm(ref)
    if nr == 0.0:
        return 0.0 if np.linalg.norm(x) == 0.0 else np.inf
    return float(np.linalg.norm(x - ref) / nr)


def tol(precision: str) -> float:
    return FP32_TOL if precision == "fp32" else BF16_TOL


def make_pair(scene, precision="fp32", ids=None, max_rays=None, rays_per_tile=0, seed_init=True,
              lr=1e-3, rays_per_tile_wide=0, split_step=False):
    """An ObjectSet with the scene's objects registered, plus the oracle states of the same
    objects (initial parameters read back from the library: the init kernel is checked against
    the oracle's own initialisation separately)."""
    import paper_2302_01838_amd as vm
    ids = list(range(scene.n_objects)) if ids is None else ids
    H = max(scene.objects[k].hidden for k in ids)
    if max_rays is None:
        max_rays = int(sum(scene.objects[k].n_rays for k in ids)) + 64
    objs = vm.ObjectSet(max_objects=len(ids), B=scene.B, hidden=scene.objects[ids[0]].hidden,
                        max_hidden=H, precision=precision, max_rays=max_rays,
                        max_samples_per_ray=max(scene.S, 1), rays_per_tile=rays_per_tile,
                        rays_per_tile_wide=rays_per_tile_wide, lr=lr, split_step=split_step)
    states = {}
    for j, k in enumerate(ids):
        ob = scene.objects[k]
        kid = objs.add(ob.norm_centre, ob.norm_scale, hidden=ob.hidden, seed=ob.seed)
        assert kid == j
        th = objs.get_state(kid, vm.STATE_PARAMS)
        # the library stores centre and scale as FP32: give the oracle the same values
        c32 = np.asarray(ob.norm_centre, np.float32).astype(np.float64)
        s32 = float(np.float32(ob.norm_scale))
        states[kid] = oracle.ObjectState(th, ob.hidden, 4, c32, s32)
    return objs, states


def remap_batch(batch, ids):
    """Rename scene object ids to library ids (registration order)."""
    lut = {k: j for j, k in enumerate(ids)}
    out = dict(batch)
    out["object_ids"] = np.asarray([lut[int(k)] for k in batch["object_ids"]], dtype=np.int32)
    return out


def near_kink_rays(states, batch, B, tau=1e-5, rnd=None):
    """Boolean mask [R] of rays whose FP64 forward puts a decision within ``tau`` of its kink.

    The gradient of the step is piecewise smooth: a ReLU mask 1[a > 0] and an L1 sign sgn(r) are
    integers decided by floating point. A decision whose argument is within rounding of zero can
    go either way in FP32; one flipped decision moves the object's gradient by a whole sample's
    contribution. A ray is near a kink when any hidden pre-activation of any of its samples has
    |a| < tau * (sum_j |W_uj h_j| + |b_u|), or a masked depth or colour residual has
    |r| < tau * (|rendered| + |target|).
    """
    offs = np.asarray(batch["ray_offsets"], np.int64)
    R, S = batch["t"].shape
    near = np.zeros(R, dtype=bool)
    for j, k in enumerate(batch["object_ids"]):
        r0, r1 = offs[j], offs[j + 1]
        if r1 == r0:
            continue
        st = states[int(k)]
        kw = {} if rnd is None else {"rnd": rnd}
        if batch.get("var") is not None:
            kw["var"] = batch["var"][r0:r1]
        fw = oracle.object_forward(st.theta, st.H, st.L, B, st.centre, st.scale,
                                   batch["rays_o"][r0:r1], batch["rays_d"][r0:r1], batch["t"][r0:r1],
                                   **kw)
        layers = oracle.unpack(np.asarray(st.theta, np.float64), st.H, st.L, fw["gamma"].shape[-1])
        h = fw["gamma"]
        amb = np.zeros((r1 - r0) * S, dtype=bool)
        for (W, b), a in zip(layers[:-1], fw["pre"]):
            scale = np.abs(h) @ np.abs(W).T + np.abs(b)
            amb |= np.any(np.abs(a) < tau * scale, axis=1)
            h = np.maximum(a, 0.0)
        ray_amb = amb.reshape(r1 - r0, S).any(axis=1)
        M = np.asarray(batch["mask"][r0:r1], np.float64) == 1.0
        D = np.asarray(batch["depth"][r0:r1], np.float64)
        C = np.asarray(batch["rgb"][r0:r1], np.float64)
        ray_amb |= M & (np.abs(fw["D"] - D) < tau * (np.abs(fw["D"]) + np.abs(D)))
        ray_amb |= M & np.any(np.abs(fw["C"] - C) < tau * (np.abs(fw["C"]) + np.abs(C)), axis=1)
        near[r0:r1] = ray_amb
    return near


def keep_rays(batch, keep):
    """The batch restricted to the rays where ``keep`` is true (CSR offsets recomputed)."""
    offs = np.asarray(batch["ray_offsets"], np.int64)
    counts = [int(np.sum(keep[offs[j]:offs[j + 1]])) for j in range(len(batch["object_ids"]))]
    out = {k: batch[k][keep] for k in ("rays_o", "rays_d", "t", "depth", "rgb", "mask")}
    if batch.get("var") is not None:
        out["var"] = batch["var"][keep]
    out["object_ids"] = batch["object_ids"].copy()
    out["ray_offsets"] = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    out["S"] = batch["S"]
    return out


def away_from_kinks(states, batch, B, tau=1e-5, rnd=None):
    """(batch without near-kink rays, number of rays dropped)."""
    near = near_kink_rays(states, batch, B, tau, rnd)
    return keep_rays(batch, ~near), int(near.sum())


def report(name, **errs):
    print(f"[parity] {name}: " + ", ".join(f"{k}={v:.3e}" for k, v in errs.items()), flush=True)


def scaled(scene, factor=10):
    """The scene with every object's ray count divided by ``factor`` (at least 1)."""
    sc = dataclasses.replace(scene, objects=[dataclasses.replace(o, n_rays=max(1, o.n_rays // factor))
                                             for o in scene.objects])
    return sc


def step_errors(objs, states, batch, precision, B):
    """One library step against the oracle on the batch without its near-kink rays. Returns
    (errors vs FP64, errors vs the oracle's BF16 mode or None, sign-unstable gradient count,
    oracle states after the step)."""
    batch, dropped = away_from_kinks(states, batch, B,
                                     rnd=oracle.bf16_round if precision == "bf16" else None)
    print(f"[parity] near-kink rays dropped: {dropped}", flush=True)
    import torch
    import paper_2302_01838_amd as vm
    db = vm.DeviceBatch(batch)
    loss = objs.step(db)
    torch.cuda.synchronize()
    st = {k: v.copy() for k, v in states.items()}
    l_ref, g_ref, _ = oracle.step(st, batch, B)
    st16 = g16 = None
    if precision == "bf16":
        st16 = {k: v.copy() for k, v in states.items()}
        _, g16, _ = oracle.step(st16, batch, B, rnd=oracle.bf16_round)
    errs = dict(loss=0.0, theta=0.0, theta_stable=0.0, m=0.0, v=0.0, grad=0.0)
    errs16 = dict(m=0.0, v=0.0, grad=0.0) if precision == "bf16" else None
    unstable = 0
    lr = objs.cfg.lr
    for j, k in enumerate(batch["object_ids"]):
        k = int(k)
        errs["loss"] = max(errs["loss"], relerr(loss[j].item(), l_ref[j]))
        th = objs.get_state(k, vm.STATE_PARAMS)
        m = objs.get_state(k, vm.STATE_ADAM_M)
        v = objs.get_state(k, vm.STATE_ADAM_V)
        g = objs.get_state(k, vm.STATE_GRAD)
        errs["theta"] = max(errs["theta"], relerr(th, st[k].theta))
        errs["m"] = max(errs["m"], relerr(m, st[k].m))
        errs["v"] = max(errs["v"], relerr(v, st[k].v))
        errs["grad"] = max(errs["grad"], relerr(g, g_ref[k]))
        # Adam's first step moves each parameter by about lr * sign(g). An element whose FP64
        # gradient lies within 10x the largest elementwise gradient error of its object is
        # "sign-unstable": its update direction is decided by rounding. Those elements are held
        # to the Adam bound (at most 2 lr apart); all others to the tolerance.
        gerr = np.max(np.abs(g.astype(np.float64) - g_ref[k]))
        uns = np.abs(g_ref[k]) < 10.0 * gerr
        if st[k].t == 1 and precision == "fp32":
            unstable += int(np.sum(uns))
            stable = ~uns
            errs["theta_stable"] = max(errs["theta_stable"], relerr(th[stable], st[k].theta[stable]))
            assert np.all(np.abs(th[uns] - st[k].theta[uns]) <= 2.0 * lr * (1 + 1e-5))
        else:
            errs["theta_stable"] = max(errs["theta_stable"], relerr(th, st[k].theta))
        if errs16 is not None:
            errs16["m"] = max(errs16["m"], relerr(m, st16[k].m))
            errs16["v"] = max(errs16["v"], relerr(v, st16[k].v))
            errs16["grad"] = max(errs16["grad"], relerr(g, g16[k]))
        assert objs.get_state(k, vm.STATE_STEP) == st[k].t
    return errs, errs16, unstable, st


def check_step(errs, errs16, precision):
    if precision == "fp32":
        for key, v in errs.items():
            if key != "theta":  # theta: the sign-unstable elements are bounded separately
                assert v <= 1e-5, key
    else:
        for key in ("loss", "theta"):
            assert errs[key] <= 2e-2
        for v in errs16.values():
            assert v <= BF16_VS_BF16_ORACLE


def snapshot(objs, ids):
    import paper_2302_01838_amd as vm
    return {k: [objs.get_state(k, w) for w in (vm.STATE_PARAMS, vm.STATE_ADAM_M, vm.STATE_ADAM_V)]
            + [objs.get_state(k, vm.STATE_STEP)] for k in ids}


def same_state(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def subbatch(batch, js):
    offs = batch["ray_offsets"]
    rows = np.concatenate([np.arange(offs[j], offs[j + 1]) for j in js]).astype(np.int64)
    counts = [offs[j + 1] - offs[j] for j in js]
    out = {k: batch[k][rows] for k in ("rays_o", "rays_d", "t", "depth", "rgb", "mask")}
    out["object_ids"] = batch["object_ids"][list(js)]
    out["ray_offsets"] = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    out["S"] = batch["S"]
    return out
