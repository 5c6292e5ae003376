"""GPU parity of hidden-16 objects, which run in the width-32 tile kernels with their weights
zero-padded to 32 units, against the FP64 oracle at hidden 16, through the C ABI.

The padding is exact: the extra units' pre-activations are exactly zero, so they never activate,
add exact zeros to every sum and get zero gradients (tests/test_padded_width_cpu.py shows it on
the oracle's arithmetic). What these tests pin is the library's side of it: the zero-padded
weight images, the optimisers reading the padded partials for the object's own parameters, the
queries staging the padded weights, and hidden-16 and hidden-32 objects sharing one launch.
Tolerances as in tests/test_gpu_parity.py (1e-5 FP32; BF16 against the oracle's BF16 mode).
"""
import dataclasses

import numpy as np
import pytest

import oracle
import scenes
from vmap_testlib import (BF16_VS_BF16_ORACLE, away_from_kinks, check_step, make_pair, relerr,
                          report, same_state, scaled, snapshot, step_errors, tol)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, never run there
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2302_01838_amd as vm  # noqa: E402


def _h16(sc, widths=None):
    """The scene with every object (or object k: widths[k]) at hidden 16."""
    objs = [dataclasses.replace(o, hidden=(widths[k] if widths else 16)) for k, o in enumerate(sc.objects)]
    return dataclasses.replace(sc, objects=objs)


SCENES = {
    "tiny_k4": lambda: _h16(scenes.make_scene("tiny_k4")),
    "k50_div10": lambda: _h16(scaled(scenes.make_scene("k50_uneven"), 10)),
}


def test_init_matches_oracle_bitwise():
    B = scenes.make_encoding_matrix(0)
    objs = vm.ObjectSet(max_objects=4, B=B, hidden=16, max_rays=256, max_samples_per_ray=8)
    for seed in (0, 1, 2 ** 40 + 7):
        k = objs.add([0.1, -0.2, 0.3], 0.5, seed=seed)
        got = objs.get_state(k, vm.STATE_PARAMS)
        want = oracle.xavier_init(seed, 16, 4, 32)
        assert got.shape == (1412,) and np.array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("scene_name", list(SCENES))
def test_train_step_parity(precision, scene_name):
    print(f"[h16] step {precision} {scene_name}", flush=True)
    sc = SCENES[scene_name]()
    objs, states = make_pair(sc, precision)
    errs, errs16, unstable, _ = step_errors(objs, states, scenes.make_batch(sc, 0), precision, sc.B)
    report(f"h16 step {precision} {scene_name} (sign-unstable={unstable})", **errs)
    if errs16:
        report(f"h16 step {precision} {scene_name} vs bf16 oracle", **errs16)
    check_step(errs, errs16, precision)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_full_size_k50_step(precision):
    """The 50-object uneven workload (16,881 rays of 20 samples) with every object at hidden 16,
    in the launch shape the benchmark uses, every object checked."""
    print(f"[h16] full-size k50 {precision}", flush=True)
    sc = _h16(scenes.make_scene("k50_uneven"))
    objs, states = make_pair(sc, precision)
    errs, errs16, unstable, _ = step_errors(objs, states, scenes.make_batch(sc, 3), precision, sc.B)
    report(f"h16 step {precision} k50 full (sign-unstable={unstable})", **errs)
    if errs16:
        report(f"h16 step {precision} k50 full vs bf16 oracle", **errs16)
    check_step(errs, errs16, precision)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_backward_parity(precision):
    print(f"[h16] backward {precision}", flush=True)
    sc = SCENES["tiny_k4"]()
    objs, states = make_pair(sc, precision)
    rnd = oracle.bf16_round if precision == "bf16" else None
    batch, dropped = away_from_kinks(states, scenes.make_batch(sc, 0), sc.B, rnd=rnd,
                                     tau_res=1e-5 if precision == "fp32" else 2.0 ** -8)
    db = vm.DeviceBatch(batch)
    up = np.linspace(0.5, 2.0, len(batch["object_ids"])).astype(np.float32)
    grad = objs.backward(db, torch.tensor(up)).cpu().numpy()
    kw = dict(apply_adam=False, upstream=up.astype(np.float64))
    _, g_ref, _ = oracle.step({k: v.copy() for k, v in states.items()}, batch, sc.B, **kw)
    _, g_b16, _ = oracle.step({k: v.copy() for k, v in states.items()}, batch, sc.B, rnd=oracle.bf16_round, **kw)
    worst = worst_b16 = 0.0
    for j, k in enumerate(batch["object_ids"]):
        P = objs.n_params[int(k)]
        assert P == 1412
        worst = max(worst, relerr(grad[j, :P], g_ref[int(k)]))
        worst_b16 = max(worst_b16, relerr(grad[j, :P], g_b16[int(k)]))
        assert not np.any(grad[j, P:]), "padding of the gradient slot must stay zero"
    report(f"h16 backward {precision} (near-kink rays dropped={dropped})", grad_vs_fp64=worst,
           grad_vs_bf16_oracle=worst_b16)
    assert (worst <= 1e-5) if precision == "fp32" else (worst_b16 <= BF16_VS_BF16_ORACLE)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_forward_and_query_parity(precision):
    print(f"[h16] forward and query {precision}", flush=True)
    sc = SCENES["tiny_k4"]()
    objs, states = make_pair(sc, precision)
    batch = scenes.make_batch(sc, 0)
    loss, depth, rgb, occ = objs.forward(vm.DeviceBatch(batch))
    torch.cuda.synchronize()
    l_ref, _, rend = oracle.step({k: v.copy() for k, v in states.items()}, batch, sc.B, apply_adam=False)
    e = dict(loss=relerr(loss.cpu().numpy(), np.asarray(l_ref)), depth=relerr(depth.cpu().numpy(), rend["D"]),
             rgb=relerr(rgb.cpu().numpy(), rend["C"]), occ=relerr(occ.cpu().numpy(), rend["O"]))
    for k in range(2):
        pts = scenes.make_points(sc, k, 300, seed=k)
        q_occ, q_rgb = objs.query(k, pts)
        st = states[k]
        o_ref, c_ref = oracle.query(st.theta, st.H, st.L, sc.B, st.centre, st.scale, pts)
        e[f"query_occ{k}"] = relerr(q_occ.cpu().numpy(), o_ref)
        e[f"query_rgb{k}"] = relerr(q_rgb.cpu().numpy(), c_ref)
    report(f"h16 forward/query {precision}", **e)
    assert max(e.values()) <= tol(precision)


@pytest.mark.parametrize("S", [1, 17])
def test_ragged_samples(S):
    print(f"[h16] ragged S={S}", flush=True)
    sc = dataclasses.replace(SCENES["tiny_k4"](), S=S, n_strat=max(1, S // 2))
    objs, states = make_pair(sc, "bf16")
    batch = scenes.make_batch(sc, 0, n_rays={0: 1, 1: 37, 2: 5, 3: 90})
    errs, errs16, _, _ = step_errors(objs, states, batch, "bf16", sc.B)
    report(f"h16 ragged S={S}", **errs)
    check_step(errs, errs16, "bf16")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_mixed_with_width32_in_one_launch(precision):
    """Hidden-16 and hidden-32 objects in one stack and one batch (one tile launch): each matches
    the oracle at its own width, and each ends bit for bit as when its width is stepped alone."""
    print(f"[h16] mixed 16/32 {precision}", flush=True)
    base = scaled(scenes.make_scene("k50_uneven"), 10)
    n = base.n_objects
    widths = [16 if k % 2 == 0 else 32 for k in range(n)]
    sc = _h16(base, widths)
    objs, states = make_pair(sc, precision)
    assert [objs.n_params[k] for k in range(n)] == [1412 if w == 16 else 4356 for w in widths]
    batch = scenes.make_batch(sc, 0)
    errs, errs16, _, _ = step_errors(objs, states, batch, precision, sc.B)
    report(f"h16 mixed {precision}", **errs)
    check_step(errs, errs16, precision)
    both, _ = make_pair(sc, precision)
    both.step(vm.DeviceBatch(batch))
    mixed = snapshot(both, range(n))
    for w in (16, 32):
        ids = [k for k in range(n) if widths[k] == w]
        alone, _ = make_pair(sc, precision)
        alone.step(vm.DeviceBatch(scenes.make_batch(sc, 0, object_ids=ids)))
        got = snapshot(alone, ids)
        assert all(same_state(got[k], mixed[k]) for k in ids), w
