"""Robustness of the training step through the C ABI: batches whose device-side ray offsets are
corrupt, the dynamic loss scaler (growth, power-of-two exactness), stop and resume from a
checkpoint (Sec. 3.2: objects stop and resume training without interference), the debug
validation of VMAP_DEBUG=1, and the per-step log.

Expected values here are the library's own results under another schedule (bitwise), the
scaler's state machine, or the state before a call that must not change it; parity with the FP64
oracle is covered by the parity tests.
"""
import json
import os

import numpy as np
import pytest

import scenes
from vmap_testlib import make_pair, remap_batch, same_state, scaled, snapshot

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, never run there
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2302_01838_amd as vm  # noqa: E402

WHAT = (vm.STATE_PARAMS, vm.STATE_ADAM_M, vm.STATE_ADAM_V, vm.STATE_GRAD)


def _same(a, b, ids, what=WHAT):
    for k in ids:
        for w in what:
            assert np.array_equal(a.get_state(k, w), b.get_state(k, w), equal_nan=True), (k, w)
        assert a.get_state(k, vm.STATE_STEP) == b.get_state(k, vm.STATE_STEP), k


def _step(objs, batch):
    db = batch if isinstance(batch, vm.DeviceBatch) else vm.DeviceBatch(batch)
    loss = objs.step(db).cpu().numpy()
    torch.cuda.synchronize()
    return loss


def _corrupt(db, kind):
    """Overwrite the batch's device offsets (the host's n_rays_total stays as it was)."""
    offs = db.ray_offsets.copy()
    n = len(offs) - 1
    if kind == "decreasing":
        offs[2] = offs[1] - 1
    elif kind == "beyond":
        offs[3] = offs[-1] + 100000
    elif kind == "last":
        offs[-1] = offs[-1] - 1
    elif kind == "first":
        offs[0] = 1
    elif kind == "huge":
        offs[n // 2] = 2 ** 31 - 1
    elif kind == "negative":
        offs[1] = -(2 ** 31)
    db.tensors["ray_offsets"].copy_(torch.as_tensor(offs.astype(np.int32)))


@pytest.mark.parametrize("split_step", [False, True])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("kind", ["decreasing", "beyond", "last", "first", "huge", "negative"])
def test_corrupt_offsets_batch_is_not_run(kind, precision, split_step):
    """A batch whose device offsets are not a CSR over its rays changes nothing: parameters,
    moments, step counts and the scaler stay bitwise as they were, its losses are 0, and
    device error bit 2 is raised. The next valid step then matches a twin that never saw it."""
    print(f"[robust] corrupt offsets {kind} {precision} split={split_step}", flush=True)
    sc = scaled(scenes.make_scene("k50_uneven"), 10)
    objs, _ = make_pair(sc, precision, split_step=split_step)
    twin, _ = make_pair(sc, precision, split_step=split_step)
    ids = range(sc.n_objects)
    first = scenes.make_batch(sc, 0)
    _step(objs, first)
    _step(twin, first)
    before = snapshot(objs, ids)
    scaler = objs.get_state(-1, vm.STATE_SCALER)
    db = vm.DeviceBatch(scenes.make_batch(sc, 1))
    _corrupt(db, kind)
    loss = _step(objs, db)
    assert np.all(loss == 0.0)
    after = snapshot(objs, ids)
    assert all(same_state(before[k], after[k]) for k in ids)
    assert objs.get_state(-1, vm.STATE_SCALER) == scaler
    assert objs.step_info()[2] & vm.DERR_OFFSETS
    good = scenes.make_batch(sc, 2)
    assert np.array_equal(_step(objs, good), _step(twin, good))
    _same(objs, twin, ids)


def test_corrupt_offsets_forward_and_graph():
    """The same check on the forward path (losses 0) and under hipGraph replay."""
    sc = scaled(scenes.make_scene("k50_uneven"), 10)
    objs, _ = make_pair(sc, "bf16")
    db = vm.DeviceBatch(scenes.make_batch(sc, 0))
    _corrupt(db, "decreasing")
    loss, _, _, _ = objs.forward(db)
    torch.cuda.synchronize()
    assert np.all(loss.cpu().numpy() == 0.0)
    assert objs.step_info()[2] & vm.DERR_OFFSETS
    objs.set_graph_mode(True)
    before = snapshot(objs, range(sc.n_objects))
    _step(objs, db)
    assert all(same_state(before[k], v) for k, v in snapshot(objs, range(sc.n_objects)).items())
    twin, _ = make_pair(sc, "bf16")
    good = scenes.make_batch(sc, 1)
    assert np.array_equal(_step(objs, good), _step(twin, good))
    _same(objs, twin, range(sc.n_objects))


def test_scaler_grows_after_good_steps_and_halves_on_overflow():
    """BF16 scaler with growth interval 2: x2 after every second good step; a non-finite object
    halves it and restarts the count (Q18 reading of the loss-scaling schedule)."""
    sc = scaled(scenes.make_scene("k50_uneven"), 10)
    objs = vm.ObjectSet(max_objects=sc.n_objects, B=sc.B, precision="bf16",
                        max_rays=int(sum(o.n_rays for o in sc.objects)) + 64,
                        max_samples_per_ray=sc.S, scale_growth_interval=2, loss_scale_init=2.0 ** 10)
    for ob in sc.objects:
        objs.add(ob.norm_centre, ob.norm_scale, seed=ob.seed)
    seen = []
    for s in range(5):
        _step(objs, scenes.make_batch(sc, s))
        seen.append(objs.get_state(-1, vm.STATE_SCALER))
    assert seen == [(2.0 ** 10, 1), (2.0 ** 11, 0), (2.0 ** 11, 1), (2.0 ** 12, 0), (2.0 ** 12, 1)]
    bad = scenes.make_batch(sc, 5)
    bad["rays_o"] = bad["rays_o"].copy()
    bad["rays_o"][int(bad["ray_offsets"][7])] = np.inf
    _step(objs, bad)
    assert objs.get_state(-1, vm.STATE_SCALER) == (2.0 ** 11, 0)
    assert objs.step_info()[1] == 1
    _step(objs, scenes.make_batch(sc, 6))
    _step(objs, scenes.make_batch(sc, 7))
    assert objs.get_state(-1, vm.STATE_SCALER) == (2.0 ** 12, 0)


@pytest.mark.parametrize("split_step", [False, True])
def test_power_of_two_scales_are_bitwise_equal(split_step):
    """Rounding to nearest even commutes with scaling by 2^k: two BF16 runs whose loss scales
    differ by a power of two (2^8 and 2^12, no overflow) give bitwise equal losses, gradients,
    parameters and moments over several steps."""
    sc = scaled(scenes.make_scene("k50_uneven"), 10)
    runs = []
    for init in (2.0 ** 8, 2.0 ** 12):
        o = vm.ObjectSet(max_objects=sc.n_objects, B=sc.B, precision="bf16",
                         max_rays=int(sum(x.n_rays for x in sc.objects)) + 64,
                         max_samples_per_ray=sc.S, loss_scale_init=init, split_step=split_step)
        for ob in sc.objects:
            o.add(ob.norm_centre, ob.norm_scale, seed=ob.seed)
        runs.append(o)
    for s in range(3):
        b = scenes.make_batch(sc, s)
        assert np.array_equal(_step(runs[0], b), _step(runs[1], b)), s
    _same(runs[0], runs[1], range(sc.n_objects))
    assert runs[0].step_info()[1] == 0 and runs[1].step_info()[1] == 0


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_checkpoint_resume_is_bitwise(tmp_path, precision):
    """N steps, save (parameters, moments, step counts, scaler), restore into a fresh context,
    M more steps: bitwise the state of N + M straight steps. One object is paused (no rays)
    across the checkpoint, and the scaler's good-step count crosses it (growth interval 3)."""
    sc = scaled(scenes.make_scene("k50_uneven"), 10)
    R = int(sum(o.n_rays for o in sc.objects)) + 64

    def fresh():
        o = vm.ObjectSet(max_objects=sc.n_objects, B=sc.B, precision=precision, max_rays=R,
                         max_samples_per_ray=sc.S, scale_growth_interval=3)
        for ob in sc.objects:
            o.add(ob.norm_centre, ob.norm_scale, seed=ob.seed)
        return o

    batches = [scenes.make_batch(sc, s, n_rays={4: 0} if s in (1, 2, 3) else None) for s in range(6)]
    straight = fresh()
    for b in batches[:4]:
        _step(straight, b)
    path = str(tmp_path / "ckpt.npz")
    straight.save(path)
    resumed = fresh()
    resumed.load(path)
    _same(straight, resumed, range(sc.n_objects), what=WHAT[:3])
    assert resumed.get_state(-1, vm.STATE_SCALER) == straight.get_state(-1, vm.STATE_SCALER)
    for b in batches[4:]:
        assert np.array_equal(_step(straight, b), _step(resumed, b))
    _same(straight, resumed, range(sc.n_objects))
    assert straight.get_state(-1, vm.STATE_SCALER) == resumed.get_state(-1, vm.STATE_SCALER)
    assert straight.get_state(4, vm.STATE_STEP) == 3 and straight.get_state(0, vm.STATE_STEP) == 6


def test_scaler_state_rejects_bad_values():
    sc = scenes.make_scene("tiny_k4")
    objs, _ = make_pair(sc, "bf16")
    for bad in [(3.0, 0), (0.0, 0), (float("inf"), 0), (2.0 ** 127, 0), (4.0, -1)]:
        with pytest.raises(vm.VmapError):
            objs.set_state(-1, vm.STATE_SCALER, bad)
    objs.set_state(-1, vm.STATE_SCALER, (2.0 ** -3, 5))
    assert objs.get_state(-1, vm.STATE_SCALER) == (2.0 ** -3, 5)


def test_debug_validation_reports_unsorted_samples_and_repeated_ids(monkeypatch):
    """With VMAP_DEBUG=1 at creation a context checks every batch on the device: a ray whose
    sample depths descend sets bit 3, an id named twice sets bit 4 (report only). A context
    created without it runs no such check."""
    sc = scenes.make_scene("tiny_k4")
    monkeypatch.setenv("VMAP_DEBUG", "1")
    dbg, _ = make_pair(sc, "fp32")
    monkeypatch.delenv("VMAP_DEBUG")
    plain, _ = make_pair(sc, "fp32")
    good = scenes.make_batch(sc, 0)
    for o in (dbg, plain):
        o.render(vm.DeviceBatch(good))
        assert o.step_info()[2] == 0
    unsorted = dict(good)
    unsorted["t"] = good["t"].copy()
    unsorted["t"][5] = unsorted["t"][5][::-1]
    for o in (dbg, plain):
        o.render(vm.DeviceBatch(unsorted))
    assert dbg.step_info()[2] == vm.DERR_T_ORDER and plain.step_info()[2] == 0
    rep = scenes.make_batch(sc, 1, object_ids=[0, 1, 2])
    rep["object_ids"] = np.asarray([0, 2, 0], dtype=np.int32)
    for o in (dbg, plain):
        o.render(vm.DeviceBatch(rep))
    assert dbg.step_info()[2] == vm.DERR_T_ORDER | vm.DERR_DUP_ID and plain.step_info()[2] == 0


def test_step_log(tmp_path):
    """The optional per-step JSON-lines log: step, per-object losses, total, loss scale,
    skipped objects, step time."""
    sc = scenes.make_scene("tiny_k4")
    path = str(tmp_path / "steps.jsonl")
    objs = vm.ObjectSet(max_objects=4, B=sc.B, precision="bf16", max_rays=1024,
                        max_samples_per_ray=sc.S, log_path=path)
    for ob in sc.objects:
        objs.add(ob.norm_centre, ob.norm_scale, seed=ob.seed)
    losses = [_step(objs, scenes.make_batch(sc, s)) for s in range(3)]
    recs = [json.loads(ln) for ln in open(path)]
    assert [r["step"] for r in recs] == [1, 2, 3]
    for r, l in zip(recs, losses):
        assert np.allclose(r["loss"], l) and abs(r["total"] - float(np.sum(l))) <= 1e-6 * abs(r["total"])
        assert r["loss_scale"] == 4096.0 and r["skipped"] == 0 and r["step_us"] > 0
