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
    objects. The oracle's initial parameters are its own seeded initialisation; the library's
    (its init kernel, from the same seed) must equal them bit for bit."""
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
        th = oracle.xavier_init(ob.seed, ob.hidden, 4, 32)
        assert np.array_equal(objs.get_state(kid, vm.STATE_PARAMS).view(np.uint32), th.view(np.uint32))
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


def near_kink_rays(states, batch, B, tau=1e-5, rnd=None, tau_res=None):
    """Boolean mask [R] of rays whose FP64 forward puts a decision within ``tau`` of its kink
    (``tau_res``, default ``tau``, for the L1 residuals).

    The gradient of the step is piecewise smooth: a ReLU mask 1[a > 0] and an L1 sign sgn(r) are
    integers decided by floating point. A decision whose argument is within rounding of zero can
    go either way in FP32; one flipped decision moves the object's gradient by a whole sample's
    contribution. A ray is near a kink when any hidden pre-activation of any of its samples has
    |a| < tau * (sum_j |W_uj h_j| + |b_u|), or a masked depth or colour residual has
    |r| < tau_res * (|rendered| + |target|).
    """
    tau_res = tau if tau_res is None else tau_res
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
        ray_amb |= M & (np.abs(fw["D"] - D) < tau_res * (np.abs(fw["D"]) + np.abs(D)))
        ray_amb |= M & np.any(np.abs(fw["C"] - C) < tau_res * (np.abs(fw["C"]) + np.abs(C)), axis=1)
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


def away_from_kinks(states, batch, B, tau=1e-5, rnd=None, tau_res=None):
    """(batch without near-kink rays, number of rays dropped)."""
    near = near_kink_rays(states, batch, B, tau, rnd, tau_res)
    return keep_rays(batch, ~near), int(near.sum())


def report(name, **errs):
    print(f"[parity] {name}: " + ", ".join(f"{k}={v:.3e}" for k, v in errs.items()), flush=True)


def scaled(scene, factor=10):
    """The scene with every object's ray count divided by ``factor`` (at least 1)."""
    sc = dataclasses.replace(scene, objects=[dataclasses.replace(o, n_rays=max(1, o.n_rays // factor))
                                             for o in scene.objects])
    return sc


def step_errors(objs, states, batch, precision, B):
    """One library step against the oracle on the batch without its near-kink rays.

    Returns (errors vs FP64, BF16 errors or None, sign-unstable gradient count, oracle states
    after the step). The BF16 errors hold, for the gradient and the Adam moments, the distance
    to the oracle's BF16 diagnostic mode (``*_b16``: same rounding points, FP64 accumulation),
    to the FP64 oracle whose ReLU decisions and L1 signs are taken by the BF16 forward
    (``*_dec``: FP64 arithmetic on the piece of the loss the BF16 forward selects) and to the
    plain FP64 oracle (``*_fp64``, reported only)."""
    # Decisions within 1e-5 of their kink, relative to the magnitude of their terms. In BF16 the
    # L1 residuals also within 2^-8 of theirs: the kernel and the oracle's BF16 mode round the same
    # values, but values that differ in their last FP32 bits (sine, cosine, sums in another order)
    # can round to neighbouring BF16 numbers, and the rendered depth and colour of a ray collect
    # such differences from all its samples; one flipped residual sign moves a whole ray's share
    # of the gradient.
    tau_res = 1e-5 if precision == "fp32" else 2.0 ** -8
    batch, dropped = away_from_kinks(states, batch, B, tau=1e-5, tau_res=tau_res,
                                     rnd=oracle.bf16_round if precision == "bf16" else None)
    print(f"[parity] near-kink rays dropped: {dropped} of {int(batch['ray_offsets'][-1]) + dropped}",
          flush=True)
    n_elems = 0
    import torch
    import paper_2302_01838_amd as vm
    db = vm.DeviceBatch(batch)
    loss = objs.step(db)
    torch.cuda.synchronize()
    st = {k: v.copy() for k, v in states.items()}
    l_ref, g_ref, _ = oracle.step(st, batch, B)
    errs = dict(loss=0.0, theta=0.0, theta_stable=0.0, m=0.0, v=0.0, grad=0.0)
    errs16 = None
    if precision == "bf16":
        st16 = {k: v.copy() for k, v in states.items()}
        _, g16, _ = oracle.step(st16, batch, B, rnd=oracle.bf16_round)
        stD = {k: v.copy() for k, v in states.items()}
        _, gD, _ = oracle.step(stD, batch, B, decide=oracle.bf16_round)
        errs16 = {f"{q}_{w}": 0.0 for q in ("grad", "m", "v") for w in ("b16", "dec", "fp64")}
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
        offs_j = batch["ray_offsets"]
        if precision == "fp32" and offs_j[j + 1] > offs_j[j]:
            # Adam moves each parameter by lr * m_hat / (sqrt(v_hat) + eps), about lr * sign(m)
            # while m is small: an element whose new first moment m* = beta1 m + (1 - beta1) g* is
            # within (1 - beta1) times the a-priori FP32 error bound of g is "sign-unstable" (at
            # the first step: |g*| within the bound; its direction is decided by rounding). Those
            # are held to the Adam bound (two updates apart at most); all others to the tolerance.
            beta1 = objs.cfg.beta1
            uns = sign_unstable(st[k].m, (1.0 - beta1) * fp32_grad_bound(states[k], batch, B, j))
            unstable += int(np.sum(uns))
            n_elems += uns.size
            stable = ~uns
            errs["theta_stable"] = max(errs["theta_stable"], relerr(th[stable], st[k].theta[stable]))
            bound = 2.0 * lr * adam_ratio_bound(st[k].t, beta1, objs.cfg.beta2) * (1 + 1e-5)
            assert np.all(np.abs(th[uns] - st[k].theta[uns]) <= bound)
        else:
            errs["theta_stable"] = max(errs["theta_stable"], relerr(th, st[k].theta))
        if errs16 is not None:
            for w, (sref, gref) in (("b16", (st16, g16)), ("dec", (stD, gD)), ("fp64", (st, g_ref))):
                errs16[f"grad_{w}"] = max(errs16[f"grad_{w}"], relerr(g, gref[k]))
                errs16[f"m_{w}"] = max(errs16[f"m_{w}"], relerr(m, sref[k].m))
                errs16[f"v_{w}"] = max(errs16[f"v_{w}"], relerr(v, sref[k].v))
        assert objs.get_state(k, vm.STATE_STEP) == st[k].t
    if n_elems:
        print(f"[parity] sign-unstable elements (a-priori FP32 bound): {unstable} of {n_elems} "
              f"({100.0 * unstable / n_elems:.2f} %)", flush=True)
    return errs, errs16, unstable, st


def check_step(errs, errs16, precision):
    if precision == "fp32":
        for key, v in errs.items():
            if key != "theta":  # theta: the sign-unstable elements are bounded separately
                assert v <= FP32_TOL, key
    else:
        for key in ("loss", "theta"):
            assert errs[key] <= BF16_TOL, key
        for key, v in errs16.items():
            if key.endswith("_b16"):
                assert v <= BF16_VS_BF16_ORACLE, key
            elif key.endswith("_dec"):
                assert v <= BF16_TOL, key


U32 = 2.0 ** -24       # unit roundoff of FP32
SIGN_MARGIN = 16.0     # sign-unstable: |g*| < SIGN_MARGIN * U32 * (magnitude of g's terms)


def grad_term_magnitudes(st, batch, B, j):
    """Per gradient element of batch object j, the magnitude of the terms its FP32 evaluation
    sums: the step's forward and backward evaluated in FP64 with every product and sum taken over
    absolute values (|W| |h| + |b| forward; the rendering adjoint's seeds and suffix sums in
    absolute value; |delta| |W| backward). An FP32 evaluation of element p carries an error of a
    modest multiple of U32 times this magnitude; where the element itself is smaller, rounding
    decides its sign. Computed from the oracle's forward only: nothing here comes from the GPU."""
    offs = np.asarray(batch["ray_offsets"], np.int64)
    r0, r1 = offs[j], offs[j + 1]
    var = None if batch.get("var") is None else batch["var"][r0:r1]
    fw = oracle.object_forward(st.theta, st.H, st.L, B, st.centre, st.scale, batch["rays_o"][r0:r1],
                               batch["rays_d"][r0:r1], batch["t"][r0:r1], var=var)
    R, S = fw["o"].shape
    layers = oracle.unpack(np.asarray(st.theta, np.float64), st.H, st.L, fw["gamma"].shape[-1])
    ha = [np.abs(fw["gamma"])]
    for (W, b), m in zip(layers[:-1], fw["masks"]):
        ha.append((ha[-1] @ np.abs(W).T + np.abs(b)) * m)
    M = np.asarray(batch["mask"][r0:r1], np.float64)
    o, c, T, P, tt = fw["o"], fw["c"], fw["T"], fw["P"], fw["t"]
    lc, lo = oracle.LAMBDA_COLOUR, oracle.LAMBDA_OCC
    # |dL/dT_i| terms: |a_D| t_i + sum_c |a_C| c_i + |a_O|
    ga = M[:, None] * np.abs(tt) + lc * M[:, None] * c.sum(-1) + lo
    later = np.cumsum((ga * T)[:, ::-1], axis=1)[:, ::-1]
    later = np.concatenate([later[:, 1:], np.zeros((R, 1))], axis=1)   # sum over j > i
    dz = np.empty((R * S, oracle.N_OUT))
    dz[:, 3] = (o * (1.0 - o) * ((1.0 - o) * ga * P[:, :S] + later)).reshape(-1)
    dz[:, :3] = (T[:, :, None] * lc * M[:, None, None] * c * (1.0 - c)).reshape(-1, 3)
    grads, delta = [], dz
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        grads.append((delta.T @ ha[li], delta.sum(0)))
        if li > 0:
            delta = (delta @ np.abs(W)) * fw["masks"][li - 1]
    grads.reverse()
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def fp32_grad_bound(st, batch, B, j):
    """A-priori FP32 error scale of each gradient element of batch object j (see
    grad_term_magnitudes): SIGN_MARGIN * U32 * the magnitude of its terms."""
    return SIGN_MARGIN * U32 * grad_term_magnitudes(st, batch, B, j)


def adam_ratio_bound(t, beta1=0.9, beta2=0.999):
    """Largest |m_hat| / sqrt(v_hat) of Adam at step t over all gradient histories (Cauchy-Schwarz
    on m_t = (1 - b1) sum_i b1^(t-i) g_i against v_t = (1 - b2) sum_i b2^(t-i) g_i^2): one update
    moves a parameter by at most lr times this (1 at t = 1, about 1.004 at t = 3)."""
    bc1, bc2 = 1.0 - beta1 ** t, 1.0 - beta2 ** t
    geo = sum((beta1 * beta1 / beta2) ** i for i in range(t))
    return (1.0 - beta1) / bc1 * np.sqrt(bc2 / (1.0 - beta2)) * np.sqrt(geo)


def sign_unstable(g_ref, bound):
    """Elements whose FP64 value lies within their a-priori FP32 error bound."""
    return np.abs(np.asarray(g_ref, np.float64)) < bound


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
