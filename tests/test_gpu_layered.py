"""GPU parity of the layered path (hidden 256, 512, 1024 in BF16) against the FP64 oracle.

These widths have no fused tile kernel: the step runs as a chain of launches over activations in
device memory (encoding, one product launch per layer forward, rendering, one launch per layer
and direction backward). Same acceptance as the BF16 tile kernels: renders, losses and
parameters after one step within 2e-2 of FP64; gradients and Adam moments within 2e-3 of the
oracle's BF16 mode (same rounding points) and within 2e-2 of FP64 arithmetic whose decisions are
taken in BF16, on the rays away from a kink. Also: ragged rays and samples per ray, objects whose
rows end around the 128-row blocks of the wide products, a stack that mixes a fused width with a
layered one, the autograd split, and the bitwise invariants.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import scenes
from vmap_testlib import (check_step, make_pair, relerr, remap_batch, report, same_state, snapshot,
                          step_errors)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, never run there
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2302_01838_amd as vm  # noqa: E402

WIDTHS = [256, 512, 1024]


def _scene(H, S=None, widths=None):
    """The tiny four-sphere scene with every object (or object k: widths[k]) of width H."""
    base = scenes.make_scene("tiny_k4")
    objs = [dataclasses.replace(o, hidden=(widths[k] if widths else H)) for k, o in enumerate(base.objects)]
    sc = dataclasses.replace(base, objects=objs)
    if S is not None:
        sc = dataclasses.replace(sc, S=S, n_strat=max(1, S // 2))
    return sc


@pytest.mark.parametrize("H", WIDTHS)
def test_layered_train_step_parity(H):
    print(f"[layered] step H={H}", flush=True)
    sc = _scene(H)
    objs, states = make_pair(sc, "bf16")
    errs, errs16, _, _ = step_errors(objs, states, scenes.make_batch(sc, 0), "bf16", sc.B)
    report(f"layered step H={H}", **errs)
    report(f"layered step H={H} vs bf16 oracle", **errs16)
    check_step(errs, errs16, "bf16")


@pytest.mark.parametrize("H", [256, 512])
def test_layered_forward_parity(H):
    sc = _scene(H)
    objs, states = make_pair(sc, "bf16")
    batch = scenes.make_batch(sc, 0)
    loss, depth, rgb, occ = objs.forward(vm.DeviceBatch(batch))
    torch.cuda.synchronize()
    l_ref, _, rend = oracle.step({k: v.copy() for k, v in states.items()}, batch, sc.B, apply_adam=False)
    errs = dict(loss=relerr(loss.cpu().numpy(), l_ref), depth=relerr(depth.cpu().numpy(), rend["D"]),
                rgb=relerr(rgb.cpu().numpy(), rend["C"]), occ=relerr(occ.cpu().numpy(), rend["O"]))
    report(f"layered forward H={H}", **errs)
    for v in errs.values():
        assert v <= 2e-2


@pytest.mark.parametrize("H,S", [(256, 17), (512, 1), (256, 64)])
def test_layered_ragged_rays(H, S):
    """Objects of 1, 7, 64 and 33 rays; S = 17 leaves 13 of 64 rows of each row tile empty, S = 1
    gives 64 one-sample rays per tile, S = 64 one ray per tile."""
    print(f"[layered] ragged H={H} S={S}", flush=True)
    sc = _scene(H, S=S)
    objs, states = make_pair(sc, "bf16")
    batch = scenes.make_batch(sc, 0, n_rays={0: 1, 1: 7, 2: 64, 3: 33})
    errs, errs16, _, _ = step_errors(objs, states, batch, "bf16", sc.B)
    report(f"layered ragged H={H} S={S}", **errs)
    check_step(errs, errs16, "bf16")


@pytest.mark.parametrize("H,S,rays", [(256, 1, {0: 127, 1: 128, 2: 129, 3: 255}),
                                      (512, 2, {0: 63, 1: 64, 2: 65, 3: 128})])
def test_layered_row_block_edges(H, S, rays):
    """Objects whose rows end just before, at and just after a multiple of 128: the wide products
    cut an object's rows into 128-row blocks regardless of ray boundaries, so the last block of
    an object holds 127, 128, 129 (and 126, 130) or 255 rows' remainders."""
    print(f"[layered] row blocks H={H} S={S} rays={rays}", flush=True)
    sc = _scene(H, S=S)
    objs, states = make_pair(sc, "bf16", max_rays=sum(rays.values()) + 64)
    batch = scenes.make_batch(sc, 0, n_rays=rays)
    errs, errs16, _, _ = step_errors(objs, states, batch, "bf16", sc.B)
    report(f"layered row blocks H={H} S={S}", **errs)
    check_step(errs, errs16, "bf16")


@pytest.mark.parametrize("H", [256, 512])
def test_layered_object_over_several_work_tiles(H):
    """An object of 10,000 rows (1,000 rays of 10 samples) has its weight gradient summed over
    three work tiles of about 4,096 rows (partials added in order by the optimiser), next to small
    objects of one work tile each."""
    print(f"[layered] work tiles H={H}", flush=True)
    sc = _scene(H)
    rays = {0: 1000, 1: 7, 2: 120, 3: 1}
    objs, states = make_pair(sc, "bf16", max_rays=sum(rays.values()) + 64)
    errs, errs16, _, _ = step_errors(objs, states, scenes.make_batch(sc, 0, n_rays=rays), "bf16", sc.B)
    report(f"layered work tiles H={H}", **errs)
    check_step(errs, errs16, "bf16")


@pytest.mark.parametrize("H", [256, 512])
def test_layered_results_independent_of_batch(H):
    """Four objects stepped alone and inside the whole 50-object uneven batch (several times the
    work tiles, so every launch grid differs) end with the same losses and states bit for bit:
    no launch shape chosen from the batch's size changes an object's sums."""
    print(f"[layered] batch independence H={H}", flush=True)
    base = scenes.make_scene("k50_uneven")
    sc = dataclasses.replace(base, objects=[dataclasses.replace(o, hidden=H) for o in base.objects])
    ids = [0, 1, 2, 3]
    objs, _ = make_pair(sc, "bf16")
    small = objs.step(vm.DeviceBatch(scenes.make_batch(sc, 0, object_ids=ids))).cpu().numpy()
    snap_small = snapshot(objs, ids)
    objs, _ = make_pair(sc, "bf16")
    full = objs.step(vm.DeviceBatch(scenes.make_batch(sc, 0))).cpu().numpy()
    snap_full = snapshot(objs, ids)
    assert np.array_equal(small.view(np.uint32), full[: len(ids)].view(np.uint32))
    assert all(same_state(snap_small[k], snap_full[k]) for k in ids)


@pytest.mark.parametrize("H", [256, 1024])
def test_layered_set_params_then_step(H):
    """Parameters set from the host (seeded perturbations well beyond one step's update) reach the
    wide products: their BF16 parameter copy is restaged on set_state, so the step matches the
    oracle run from the same parameters (a stale copy would run the initial weights)."""
    print(f"[layered] set params H={H}", flush=True)
    sc = _scene(H)
    objs, states = make_pair(sc, "bf16")
    rng = np.random.default_rng(23)
    for k, st in states.items():
        th = (st.theta + 0.3 * np.abs(st.theta).mean() * rng.standard_normal(st.theta.shape)).astype(np.float32)
        objs.set_state(k, vm.STATE_PARAMS, th)
        st.theta = th.astype(np.float64)
    errs, errs16, _, _ = step_errors(objs, states, scenes.make_batch(sc, 0), "bf16", sc.B)
    report(f"layered set params H={H}", **errs)
    check_step(errs, errs16, "bf16")


def test_layered_with_fused_width_in_one_step():
    """Hidden-32 objects (fused tile kernel) and hidden-256 objects (layered path) in one batch."""
    sc = _scene(0, widths=[32, 256, 32, 256])
    objs, states = make_pair(sc, "bf16")
    assert objs.cfg.max_hidden == 256
    errs, errs16, _, _ = step_errors(objs, states, scenes.make_batch(sc, 0), "bf16", sc.B)
    report("layered + fused widths", **errs)
    check_step(errs, errs16, "bf16")


def test_layered_backward_with_upstream_weights():
    """vmap_backward (the autograd split): gradient of sum_j w_j L_j against the BF16 oracle."""
    sc = _scene(256)
    objs, states = make_pair(sc, "bf16")
    from vmap_testlib import away_from_kinks
    batch, _ = away_from_kinks(states, scenes.make_batch(sc, 0), sc.B, rnd=oracle.bf16_round,
                               tau_res=2.0 ** -8)
    up = np.asarray([0.5, 1.0, 1.5, 2.0], np.float32)
    grad = objs.backward(vm.DeviceBatch(batch), torch.tensor(up)).cpu().numpy()
    _, g16, _ = oracle.step({k: v.copy() for k, v in states.items()}, batch, sc.B, apply_adam=False,
                            upstream=up.astype(np.float64), rnd=oracle.bf16_round)
    worst = 0.0
    for j, k in enumerate(batch["object_ids"]):
        P = objs.n_params[int(k)]
        worst = max(worst, relerr(grad[j, :P], g16[int(k)]))
        assert not np.any(grad[j, P:])
    report("layered backward H=256 vs bf16 oracle", grad=worst)
    assert worst <= 2e-3


def test_layered_bitwise_invariants():
    """Repeatable, independent of the other objects (a permuted batch gives the permuted
    results), and a paused object (no rays) keeps its state bit for bit."""
    sc = _scene(256)
    ids = list(range(4))
    batch = scenes.make_batch(sc, 0)
    runs = []
    for _ in range(2):
        objs, _ = make_pair(sc, "bf16")
        loss = objs.step(vm.DeviceBatch(batch)).cpu().numpy()
        runs.append((loss, snapshot(objs, ids)))
    assert np.array_equal(runs[0][0], runs[1][0])
    assert all(same_state(runs[0][1][k], runs[1][1][k]) for k in ids)
    perm = [2, 0, 3, 1]
    offs = batch["ray_offsets"]
    rows = np.concatenate([np.arange(offs[j], offs[j + 1]) for j in perm])
    pb = {k: batch[k][rows] for k in ("rays_o", "rays_d", "t", "depth", "rgb", "mask")}
    pb["object_ids"] = batch["object_ids"][perm]
    pb["ray_offsets"] = np.concatenate([[0], np.cumsum([offs[j + 1] - offs[j] for j in perm])]).astype(np.int32)
    pb["S"] = batch["S"]
    objs, _ = make_pair(sc, "bf16")
    lp = objs.step(vm.DeviceBatch(pb)).cpu().numpy()
    assert np.array_equal(lp, runs[0][0][perm])
    sp = snapshot(objs, ids)
    assert all(same_state(sp[k], runs[0][1][k]) for k in ids)
    objs, _ = make_pair(sc, "bf16")
    before = snapshot(objs, [1])[1]
    objs.step(vm.DeviceBatch(scenes.make_batch(sc, 0, n_rays={1: 0})))
    after = snapshot(objs, ids)
    assert same_state(before, after[1]) and after[1][3] == 0
    for k in (0, 2, 3):
        assert same_state(after[k], runs[0][1][k])


def test_layered_width_rules():
    """One layered width per stack; layered widths need a layered max_hidden; BF16 only; no point
    queries."""
    sc = _scene(256)
    objs = vm.ObjectSet(max_objects=4, B=sc.B, hidden=256, precision="bf16", max_rays=512,
                        max_samples_per_ray=sc.S, max_hidden=512)
    ob = sc.objects[0]
    objs.add(ob.norm_centre, ob.norm_scale, hidden=256, seed=1)
    with pytest.raises(vm.VmapError):
        objs.add(ob.norm_centre, ob.norm_scale, hidden=512, seed=2)
    with pytest.raises(vm.VmapError):
        objs.query(0, np.zeros((4, 3), np.float32))
    with pytest.raises(vm.VmapError):
        vm.ObjectSet(max_objects=4, B=sc.B, hidden=256, precision="fp32", max_rays=512,
                     max_samples_per_ray=sc.S)
