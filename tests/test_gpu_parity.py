"""GPU parity of libvmap against the FP64 oracle, through the C ABI.

Each case builds the library's object stack and the oracle's twin from one seeded scene, runs the
same batch through both, and compares per (object, tensor) with the norm-wise relative error
||x - x*|| / ||x*||: 1e-5 for FP32; 2e-2 for BF16 renders, losses and parameters after a step.

BF16 gradients and Adam moments are compared with the oracle's BF16 diagnostic mode (FP64
arithmetic on operands rounded to BF16 at the same places as the kernels) within 2e-3, and their
distance to the pure FP64 gradient is reported. The loss is piecewise smooth (L1 residuals,
ReLU): BF16 operands move forward values by ~5e-4, which flips ReLU masks and L1 signs of the
samples closest to a kink, so the BF16 gradient differs from the FP64 one by up to ~10 % at
initialisation whatever the accumulation precision. Bitwise invariants (permutation, zero-ray
objects, batch split, determinism, graph replay) compare the library with itself.

Gradient comparisons first drop the rays that put a ReLU pre-activation or an L1 residual within
1e-5 (relative to the magnitude of its terms) of its kink: such a decision is an integer decided
by floating point, FP32 and FP64 may take it differently, and one flip moves the gradient by a
whole sample's contribution (seen at full size: one layer-1 unit of one sample, 1.7e-3 of the
object's gradient norm). The number of dropped rays is reported.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import scenes
from vmap_testlib import (BF16_VS_BF16_ORACLE, check_step, make_pair, relerr, remap_batch, report,
                          same_state, scaled, snapshot, step_errors, subbatch, tol, away_from_kinks)


torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, never run there
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2302_01838_amd as vm  # noqa: E402


SCENES = {
    "tiny_k4": lambda: scenes.make_scene("tiny_k4"),
    "k50_div10": lambda: scaled(scenes.make_scene("k50_uneven"), 10),
}


def _oracle_forward(states, batch, B):
    st = {k: v.copy() for k, v in states.items()}
    return oracle.step(st, batch, B, apply_adam=False)


# ------------------------------------------------------------------------------------ init

@pytest.mark.parametrize("H", [32, 64])
def test_init_matches_oracle_bitwise(H):
    B = scenes.make_encoding_matrix(0)
    objs = vm.ObjectSet(max_objects=4, B=B, hidden=H, max_rays=256, max_samples_per_ray=8)
    for seed in (0, 1, 2 ** 40 + 7, 2 ** 64 - 1):
        k = objs.add([0.1, -0.2, 0.3], 0.5, seed=seed)
        got = objs.get_state(k, vm.STATE_PARAMS)
        want = oracle.xavier_init(seed, H, 4, 32)
        assert got.dtype == np.float32 and np.array_equal(got.view(np.uint32), want.view(np.uint32))
        assert objs.get_state(k, vm.STATE_STEP) == 0
        assert not np.any(objs.get_state(k, vm.STATE_ADAM_M))


# ------------------------------------------------------------------------------------ query

@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("n", [1, 63, 64, 1000])
def test_query_parity(precision, n):
    sc = scenes.make_scene("tiny_k4")
    objs, states = make_pair(sc, precision)
    for k in range(2):
        pts = scenes.make_points(sc, k, n, seed=n)
        occ, rgb = objs.query(k, pts)
        st = states[k]
        o_ref, c_ref = oracle.query(st.theta, st.H, st.L, sc.B, st.centre, st.scale, pts)
        e1 = relerr(occ.cpu().numpy(), o_ref)
        e2 = relerr(rgb.cpu().numpy(), c_ref)
        report(f"query {precision} n={n} k={k}", occ=e1, rgb=e2)
        assert e1 <= tol(precision) and e2 <= tol(precision)


# ------------------------------------------------------------------------------------ forward

@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("scene_name", list(SCENES))
def test_forward_parity(precision, scene_name):
    sc = SCENES[scene_name]()
    objs, states = make_pair(sc, precision)
    batch = scenes.make_batch(sc, 0)
    db = vm.DeviceBatch(batch)
    loss, depth, rgb, occ = objs.forward(db)
    depth_r, rgb_r, occ_r = objs.render(db)
    torch.cuda.synchronize()
    l_ref, _, rend = _oracle_forward(states, batch, sc.B)
    offs = batch["ray_offsets"]
    worst = dict(loss=0.0, depth=0.0, rgb=0.0, occ=0.0)
    for j in range(len(batch["object_ids"])):
        sl = slice(offs[j], offs[j + 1])
        worst["loss"] = max(worst["loss"], relerr(loss[j].item(), l_ref[j]))
        worst["depth"] = max(worst["depth"], relerr(depth.cpu().numpy()[sl], rend["D"][sl]))
        worst["rgb"] = max(worst["rgb"], relerr(rgb.cpu().numpy()[sl], rend["C"][sl]))
        worst["occ"] = max(worst["occ"], relerr(occ.cpu().numpy()[sl], rend["O"][sl]))
    report(f"forward {precision} {scene_name}", **worst)
    for v in worst.values():
        assert v <= tol(precision)
    # rendering without targets gives the same renders, bit for bit
    assert torch.equal(depth, depth_r) and torch.equal(rgb, rgb_r) and torch.equal(occ, occ_r)


# ------------------------------------------------------------------------------------ backward

@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("scene_name", list(SCENES))
def test_backward_parity(precision, scene_name):
    sc = SCENES[scene_name]()
    objs, states = make_pair(sc, precision)
    rnd = oracle.bf16_round if precision == "bf16" else None
    batch, dropped = away_from_kinks(states, scenes.make_batch(sc, 0), sc.B, rnd=rnd,
                                     tau_res=1e-5 if precision == "fp32" else 2.0 ** -8)
    db = vm.DeviceBatch(batch)
    n = len(batch["object_ids"])
    up = np.linspace(0.5, 2.0, n).astype(np.float32)
    grad = objs.backward(db, torch.tensor(up)).cpu().numpy()
    _, g_ref, _ = oracle.step({k: v.copy() for k, v in states.items()}, batch, sc.B,
                              apply_adam=False, upstream=up.astype(np.float64))
    if precision == "bf16":
        _, g_b16, _ = oracle.step({k: v.copy() for k, v in states.items()}, batch, sc.B,
                                  apply_adam=False, upstream=up.astype(np.float64),
                                  rnd=oracle.bf16_round)
    worst = worst_b16 = 0.0
    for j, k in enumerate(batch["object_ids"]):
        P = objs.n_params[int(k)]
        worst = max(worst, relerr(grad[j, :P], g_ref[int(k)]))
        if precision == "bf16":
            worst_b16 = max(worst_b16, relerr(grad[j, :P], g_b16[int(k)]))
        assert not np.any(grad[j, P:]), "padding of the gradient slot must stay zero"
    report(f"backward {precision} {scene_name} (near-kink rays dropped={dropped})",
            grad_vs_fp64=worst, grad_vs_bf16_oracle=worst_b16)
    if precision == "fp32":
        assert worst <= 1e-5
    else:
        assert worst_b16 <= BF16_VS_BF16_ORACLE


# ------------------------------------------------------------------------------------ full step

@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("scene_name", list(SCENES))
def test_train_step_parity(precision, scene_name):
    sc = SCENES[scene_name]()
    objs, states = make_pair(sc, precision)
    batch = scenes.make_batch(sc, 0)
    errs, errs16, unstable, _ = step_errors(objs, states, batch, precision, sc.B)
    report(f"step {precision} {scene_name} (sign-unstable={unstable})", **errs)
    if errs16:
        report(f"step {precision} {scene_name} vs bf16 oracle", **errs16)
    check_step(errs, errs16, precision)


def test_full_size_k50_fp32_step():
    """The paper-scale workload (50 objects, 60-600 rays, 20 samples) in the launch shape the
    benchmark uses, every object checked."""
    sc = scenes.make_scene("k50_uneven")
    objs, states = make_pair(sc, "fp32")
    batch = scenes.make_batch(sc, 3)
    errs, _, unstable, _ = step_errors(objs, states, batch, "fp32", sc.B)
    report(f"step fp32 k50 full (sign-unstable={unstable})", **errs)
    check_step(errs, None, "fp32")


def test_full_size_k50_bf16_step():
    sc = scenes.make_scene("k50_uneven")
    objs, states = make_pair(sc, "bf16")
    batch = scenes.make_batch(sc, 3)
    errs, errs16, unstable, _ = step_errors(objs, states, batch, "bf16", sc.B)
    report("step bf16 k50 full", **errs)
    report("step bf16 k50 full vs bf16 oracle", **errs16)
    check_step(errs, errs16, "bf16")


# ------------------------------------------------------------------------------------ edge cases

# The rendering scans run per ray over lanes in rows of 16: besides the extremes, ray lengths whose
# rays cross rows at odd places (7, 13), span two rows from an odd start (17, 18) or three rows
# (31: rays at lanes 0 and 31; 33: one ray over lanes 0-32).
@pytest.mark.parametrize("S", [1, 3, 7, 13, 17, 18, 31, 32, 33, 64])
def test_samples_per_ray_edges(S):
    base = scenes.make_scene("tiny_k4")
    sc = dataclasses.replace(base, S=S, n_strat=max(1, S // 2))
    objs, states = make_pair(sc, "fp32")
    batch = scenes.make_batch(sc, 0, n_rays={0: 1, 1: 7, 2: 64, 3: 33})
    errs, _, unstable, _ = step_errors(objs, states, batch, "fp32", sc.B)
    report(f"step fp32 S={S}", **errs)
    check_step(errs, None, "fp32")


def test_empty_batch_is_a_no_op():
    sc = scenes.make_scene("tiny_k4")
    objs, states = make_pair(sc, "fp32")
    batch = scenes.make_batch(sc, 0, object_ids=[])
    db = vm.DeviceBatch(batch)
    objs.step(db)
    torch.cuda.synchronize()
    for k in range(4):
        assert np.array_equal(objs.get_state(k, vm.STATE_PARAMS), states[k].theta.astype(np.float32))


# ------------------------------------------------------------------------------------ invariants

@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_bitwise_invariants(precision):
    sc = scaled(scenes.make_scene("k50_uneven"), 10)
    ids = list(range(6))
    batch = scenes.make_batch(sc, 0, object_ids=ids)
    sub = lambda js: subbatch(batch, js)
    # reference: one step of all six objects
    objs, _ = make_pair(sc, precision, ids=ids)
    l_all = objs.step(vm.DeviceBatch(batch)).cpu().numpy()
    ref = snapshot(objs, ids)
    # determinism: the same step again from the same start
    objs2, _ = make_pair(sc, precision, ids=ids)
    l2 = objs2.step(vm.DeviceBatch(batch)).cpu().numpy()
    assert np.array_equal(l2, l_all)
    s2 = snapshot(objs2, ids)
    assert all(same_state(ref[k], s2[k]) for k in ids)
    # permutation of the batch's objects permutes the results
    perm = [3, 0, 5, 1, 4, 2]
    objs3, _ = make_pair(sc, precision, ids=ids)
    l3 = objs3.step(vm.DeviceBatch(sub(perm))).cpu().numpy()
    assert np.array_equal(l3, l_all[perm])
    s3 = snapshot(objs3, ids)
    assert all(same_state(ref[k], s3[k]) for k in ids)
    # batch split: {0,1,2} then {3,4,5}
    objs4, _ = make_pair(sc, precision, ids=ids)
    la = objs4.step(vm.DeviceBatch(sub([0, 1, 2]))).cpu().numpy()
    lb = objs4.step(vm.DeviceBatch(sub([3, 4, 5]))).cpu().numpy()
    assert np.array_equal(np.concatenate([la, lb]), l_all)
    s4 = snapshot(objs4, ids)
    assert all(same_state(ref[k], s4[k]) for k in ids)
    # zero rays: object 2 is paused, the others are unaffected
    objs5, _ = make_pair(sc, precision, ids=ids)
    before = snapshot(objs5, [2])[2]
    zb = scenes.make_batch(sc, 0, object_ids=ids, n_rays={2: 0})
    l5 = objs5.step(vm.DeviceBatch(zb)).cpu().numpy()
    assert l5[2] == 0.0
    s5 = snapshot(objs5, ids)
    assert same_state(before, s5[2]) and s5[2][3] == 0
    for k in (0, 1, 3, 4, 5):
        assert same_state(ref[k], s5[k])


def test_graph_replay_matches_plain_launches():
    sc = scaled(scenes.make_scene("k50_uneven"), 10)
    batch = scenes.make_batch(sc, 0)
    db = vm.DeviceBatch(batch)
    objs, _ = make_pair(sc, "bf16")
    objs_g, _ = make_pair(sc, "bf16")
    objs_g.set_graph_mode(True)
    for step in range(3):
        l1 = objs.step(db).cpu().numpy()
        l2 = objs_g.step(db).cpu().numpy()
        torch.cuda.synchronize()
        assert np.array_equal(l1, l2), step
    for k in range(sc.n_objects):
        assert np.array_equal(objs.get_state(k, vm.STATE_PARAMS), objs_g.get_state(k, vm.STATE_PARAMS))
    assert objs.step_info() == objs_g.step_info()


def test_autograd_function_matches_train_step():
    sc = scenes.make_scene("tiny_k4")
    batch = scenes.make_batch(sc, 0)
    db = vm.DeviceBatch(batch)
    objs, _ = make_pair(sc, "fp32")
    objs2, _ = make_pair(sc, "fp32")
    token = torch.zeros(db.n_objects, objs.p_stride, device="cuda", requires_grad=True)
    loss = vm.RenderLoss.apply(token, objs, db)
    loss.sum().backward()
    objs.adam_step(db)
    l2 = objs2.step(db)
    torch.cuda.synchronize()
    assert torch.equal(loss.detach(), l2)
    for k in range(4):
        assert np.array_equal(objs.get_state(k, vm.STATE_PARAMS), objs2.get_state(k, vm.STATE_PARAMS))
        P = objs.n_params[k]
        assert np.array_equal(token.grad[k, :P].cpu().numpy(), objs2.get_state(k, vm.STATE_GRAD))


def test_invalid_object_id_raises_device_flag():
    sc = scenes.make_scene("tiny_k4")
    objs, _ = make_pair(sc, "fp32", ids=[0, 1])
    batch = remap_batch(scenes.make_batch(sc, 0, object_ids=[0, 1]), [0, 1])
    batch["object_ids"] = np.asarray([0, 7], dtype=np.int32)   # 7 is beyond max_objects
    before = objs.get_state(0, vm.STATE_PARAMS)
    objs.step(vm.DeviceBatch(batch))
    scale, skipped, err = objs.step_info()
    assert err == 1
    assert not np.array_equal(before, objs.get_state(0, vm.STATE_PARAMS))


@pytest.mark.parametrize("rpt,waves,grid", [(1, 4, 0), (5, 2, 0), (0, 4, 7), (0, 1, 3)])
def test_launch_shapes(rpt, waves, grid):
    """Tiles of one ray, two- and one-wave blocks, and persistent grids smaller than the tile
    count (blocks loop over tiles of several objects and restage weights)."""
    sc = SCENES["k50_div10"]()
    objs, states = make_pair(sc, "fp32", rays_per_tile=rpt)
    objs.set_launch(waves, grid)
    batch = scenes.make_batch(sc, 0)
    errs, _, unstable, _ = step_errors(objs, states, batch, "fp32", sc.B)
    report(f"step fp32 rays_per_tile={rpt} waves={waves} grid={grid}", **errs)
    check_step(errs, None, "fp32")


@pytest.mark.parametrize("waves,rpt", [(8, 0), (8, 72), (6, 0), (5, 0)])
def test_bf16_wide_workgroups(waves, rpt):
    """BF16 workgroups of five to eight waves (two or four gradient copies in the end-of-tile
    reduction, waves adding in two or three turns) against the oracle's BF16 bound."""
    sc = SCENES["k50_div10"]()
    objs, states = make_pair(sc, "bf16", rays_per_tile=rpt)
    objs.set_launch(waves, 0)
    batch = scenes.make_batch(sc, 0)
    errs, errs16, _, _ = step_errors(objs, states, batch, "bf16", sc.B)
    report(f"step bf16 rays_per_tile={rpt} waves={waves}", **errs)
    report(f"step bf16 rays_per_tile={rpt} waves={waves} vs bf16 oracle", **errs16)
    check_step(errs, errs16, "bf16")


def test_fp32_rejects_eight_waves():
    """FP32 tile kernels need more than 256 registers per lane: at most four waves per block."""
    sc = scenes.make_scene("tiny_k4")
    objs, _ = make_pair(sc, "fp32")
    with pytest.raises(vm.VmapError):
        objs.set_launch(8, 0)
    objs.set_launch(4, 0)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_grid_size_does_not_change_results(precision):
    sc = SCENES["k50_div10"]()
    batch = scenes.make_batch(sc, 0)
    db = vm.DeviceBatch(batch)
    out = []
    for grid in (0, 5, 64):
        objs, _ = make_pair(sc, precision)
        objs.set_launch(4, grid)
        loss = objs.step(db).cpu().numpy()
        out.append((loss, [objs.get_state(k, vm.STATE_PARAMS) for k in range(sc.n_objects)]))
    for loss, th in out[1:]:
        assert np.array_equal(loss, out[0][0])
        assert all(np.array_equal(a, b) for a, b in zip(th, out[0][1]))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_graph_replay_over_changing_batches(precision):
    """One captured graph serves batches of the same shape in different buffers."""
    sc = scaled(scenes.make_scene("k50_uneven"), 10)
    dbs = [vm.DeviceBatch(scenes.make_batch(sc, step)) for step in range(4)]
    objs, _ = make_pair(sc, precision)
    objs_g, _ = make_pair(sc, precision)
    objs_g.set_graph_mode(True)
    for db in dbs:
        l1 = objs.step(db).cpu().numpy()
        l2 = objs_g.step(db).cpu().numpy()
        assert np.array_equal(l1, l2)
    torch.cuda.synchronize()
    for k in range(sc.n_objects):
        for w in (vm.STATE_PARAMS, vm.STATE_ADAM_M, vm.STATE_ADAM_V):
            assert np.array_equal(objs.get_state(k, w), objs_g.get_state(k, w))
        assert objs.get_state(k, vm.STATE_STEP) == objs_g.get_state(k, vm.STATE_STEP) == 4


@pytest.mark.parametrize("S,n_strat", [(10, 5), (20, 10), (1, 1), (1, 0), (33, 16), (64, 32)])
def test_depth_guided_sampling_matches_oracle(S, n_strat):
    """On-device Eqs. 1-2 against the oracle's sampler: same counter-based uniforms, FP64
    arithmetic on both sides, FP32 output; sorted per ray."""
    rng = np.random.default_rng(S)
    R = 3001
    tn = rng.uniform(0.3, 1.0, R).astype(np.float32)
    tf = (tn + rng.uniform(0.5, 3.0, R)).astype(np.float32)
    depth = np.where(rng.uniform(size=R) < 0.8, rng.uniform(tn + 0.1, tf), 0.0).astype(np.float32)
    sc = scenes.make_scene("tiny_k4")
    objs = vm.ObjectSet(max_objects=1, B=sc.B, hidden=32, max_rays=16, max_samples_per_ray=8)
    seed = 0x1234_5678_9ABC + S
    t = objs.sample_rays(tn, tf, depth, S, n_strat, sigma=0.03, seed=seed).cpu().numpy()
    ref = oracle.depth_guided_samples(tn, tf, depth, S, n_strat, 0.03, seed)
    assert np.all(np.diff(t, axis=1) >= 0)
    np.testing.assert_allclose(t, ref, rtol=2.5e-7, atol=0)
    report(f"sampling S={S} n_strat={n_strat}", max_rel=float(np.max(np.abs(t - ref) / np.abs(ref))))
    # into a given tensor (a batch's t): the same values, bit for bit
    out = torch.full((R, S), float("nan"), device="cuda")
    got = objs.sample_rays(tn, tf, depth, S, n_strat, sigma=0.03, seed=seed, out=out)
    assert got is out and np.array_equal(out.cpu().numpy().view(np.uint32), t.view(np.uint32))


# ------------------------------------------------------------------------ integrated encoding

@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("scene_name", list(SCENES))
def test_integrated_encoding_step_parity(precision, scene_name):
    """Samples standing for Gaussians as wide as a 0.02 rad pixel footprint: every feature is
    attenuated by exp(-var |b|^2 / 2) in the object frame (factors down to ~0.2 here)."""
    sc = SCENES[scene_name]()
    objs, states = make_pair(sc, precision)
    batch = scenes.make_batch(sc, 0, pixel_radius=0.02)
    errs, errs16, unstable, _ = step_errors(objs, states, batch, precision, sc.B)
    report(f"ipe step {precision} {scene_name} (sign-unstable={unstable})", **errs)
    if errs16:
        report(f"ipe step {precision} {scene_name} vs bf16 oracle", **errs16)
    check_step(errs, errs16, precision)
    # the renders differ from the point-sample encoding's
    objs2, _ = make_pair(sc, precision)
    db_ipe = vm.DeviceBatch(batch)
    plain = dict(batch)
    plain.pop("var")
    d1 = objs2.render(db_ipe)[0]
    d2 = objs2.render(vm.DeviceBatch(plain))[0]
    assert not torch.equal(d1, d2)
