"""Weight images of width-32 (and zero-padded width-16) objects and the BF16 parameter copies of
wide layered-path objects, through the C ABI.

The tile kernel stages a width-32 object's weights by copying its weight image: the object's
parameters already in the byte layout of the LDS staging (BF16 with transposed copies and bias
pieces, or FP32). The image is written whole when parameters are set (object added,
vmap_set_state) and per parameter by the optimiser after each update. These tests train one
object set normally and a twin whose images are rewritten whole from its parameters after every
update (a set_state of each object's own parameters); every loss, render and state must agree
bitwise, so the incremental image writes put every parameter where the whole staging does.
"""
import dataclasses

import numpy as np
import pytest

import scenes
from vmap_testlib import make_pair, scaled

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, never run there
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2302_01838_amd as vm  # noqa: E402

WHAT = (vm.STATE_PARAMS, vm.STATE_ADAM_M, vm.STATE_ADAM_V, vm.STATE_GRAD)


def _restage(objs, ids):
    for k in ids:
        objs.set_state(k, vm.STATE_PARAMS, objs.get_state(k, vm.STATE_PARAMS))


def _same(a, b, ids):
    for k in ids:
        for w in WHAT:
            assert np.array_equal(a.get_state(k, w), b.get_state(k, w)), (k, w)
        assert a.get_state(k, vm.STATE_STEP) == b.get_state(k, vm.STATE_STEP)


@pytest.mark.parametrize("H", [32, 16])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_images_after_training_steps_match_whole_staging(precision, H):
    """Hidden 16 keeps the zero-padded width-32 image: the optimiser writes its parameters into
    their padded slots and leaves the padding zero."""
    sc = scaled(scenes.make_scene("k50_uneven"), 10)
    sc = dataclasses.replace(sc, objects=[dataclasses.replace(o, hidden=H) for o in sc.objects])
    ids = range(sc.n_objects)
    inc, _ = make_pair(sc, precision)
    whole, _ = make_pair(sc, precision)
    for s in range(3):
        db = vm.DeviceBatch(scenes.make_batch(sc, s))
        l1 = inc.step(db).cpu().numpy()
        l2 = whole.step(db).cpu().numpy()
        torch.cuda.synchronize()
        print(f"[image] {precision} H={H} step {s}: loss sum {l1.sum():.6g}", flush=True)
        assert np.array_equal(l1, l2), s
        _restage(whole, ids)
    _same(inc, whole, ids)
    db = vm.DeviceBatch(scenes.make_batch(sc, 3))
    for a, b in zip(inc.forward(db), whole.forward(db)):
        assert torch.equal(a, b)


def test_hidden128_image_after_training_steps_matches_whole_staging():
    """The BF16 image of a hidden-128 object (the room's background width, read by the
    cooperative kernel from device memory) is kept by the optimiser as well, not restaged per
    step."""
    sc = scenes.make_scene("tiny_k4")
    sc = dataclasses.replace(sc, objects=[dataclasses.replace(o, hidden=(128 if k == 1 else 32))
                                          for k, o in enumerate(sc.objects)])
    inc, _ = make_pair(sc, "bf16")
    whole, _ = make_pair(sc, "bf16")
    for s in range(3):
        db = vm.DeviceBatch(scenes.make_batch(sc, s))
        l1 = inc.step(db).cpu().numpy()
        l2 = whole.step(db).cpu().numpy()
        torch.cuda.synchronize()
        print(f"[image] hidden 128 step {s}: loss sum {l1.sum():.6g}", flush=True)
        assert np.array_equal(l1, l2), s
        _restage(whole, range(4))
    _same(inc, whole, range(4))
    pts = scenes.make_points(sc, 1, 500, seed=3)
    for a, b in zip(inc.query(1, pts), whole.query(1, pts)):
        assert torch.equal(a, b)


@pytest.mark.parametrize("H", [32, 16])
def test_images_after_autograd_adam_step(H):
    """The autograd split's Adam kernel keeps the images current as well (hidden 16: the padded
    slots of its width-32 image)."""
    sc = scenes.make_scene("tiny_k4")
    sc = dataclasses.replace(sc, objects=[dataclasses.replace(o, hidden=H) for o in sc.objects])
    inc, _ = make_pair(sc, "bf16")
    whole, _ = make_pair(sc, "bf16")
    db = vm.DeviceBatch(scenes.make_batch(sc, 0))
    for o in (inc, whole):
        o.backward(db, torch.ones(db.n_objects, device="cuda"))
        o.adam_step(db)
    torch.cuda.synchronize()
    _restage(whole, range(4))
    db1 = vm.DeviceBatch(scenes.make_batch(sc, 1))
    l1 = inc.step(db1).cpu().numpy()
    l2 = whole.step(db1).cpu().numpy()
    assert np.array_equal(l1, l2)
    _same(inc, whole, range(4))


def test_set_state_restages_the_image():
    """Parameters written through vmap_set_state are what the next step trains: a set whose
    objects were added with random weights and then given new parameters trains exactly like a
    set whose objects were added with those parameters."""
    sc = scenes.make_scene("tiny_k4")
    a, _ = make_pair(sc, "bf16")
    rng = np.random.default_rng(5)
    new = {}
    for k in range(4):
        th = a.get_state(k, vm.STATE_PARAMS)
        new[k] = (th + rng.standard_normal(th.shape).astype(np.float32) * np.float32(0.05)).astype(np.float32)
        a.set_state(k, vm.STATE_PARAMS, new[k])
    b = vm.ObjectSet(max_objects=4, B=sc.B, precision="bf16", max_rays=a.cfg.max_rays,
                     max_samples_per_ray=sc.S)
    for k in range(4):
        ob = sc.objects[k]
        assert b.add(ob.norm_centre, ob.norm_scale, seed=ob.seed, init=new[k]) == k
    db = vm.DeviceBatch(scenes.make_batch(sc, 0))
    la = a.step(db).cpu().numpy()
    lb = b.step(db).cpu().numpy()
    assert np.array_equal(la, lb)
    _same(a, b, range(4))


def _layered_scene(H):
    import dataclasses
    base = scenes.make_scene("tiny_k4")
    return dataclasses.replace(base, objects=[dataclasses.replace(o, hidden=H) for o in base.objects])


@pytest.mark.parametrize("H", [256, 1024])
def test_layered_bf16_copy_after_steps_matches_whole_staging(H):
    """The layered path's wide products read W from a BF16 copy of each object's parameters,
    which the optimiser writes with every update (four at a time in the wide optimiser): after
    each training step, and after an autograd-split Adam step, a twin whose copies are rebuilt
    whole from its parameters trains, renders and stores bit for bit alike."""
    sc = _layered_scene(H)
    ids = range(4)
    inc, _ = make_pair(sc, "bf16")
    whole, _ = make_pair(sc, "bf16")
    for s in range(3):
        db = vm.DeviceBatch(scenes.make_batch(sc, s))
        l1 = inc.step(db).cpu().numpy()
        l2 = whole.step(db).cpu().numpy()
        torch.cuda.synchronize()
        print(f"[image] layered H={H} step {s}: loss sum {l1.sum():.6g}", flush=True)
        assert np.array_equal(l1, l2), s
        _restage(whole, ids)
    db = vm.DeviceBatch(scenes.make_batch(sc, 3))
    for o in (inc, whole):
        o.backward(db, torch.ones(db.n_objects, device="cuda"))
        o.adam_step(db)
    torch.cuda.synchronize()
    _restage(whole, ids)
    _same(inc, whole, ids)
    db = vm.DeviceBatch(scenes.make_batch(sc, 4))
    for a, b in zip(inc.forward(db), whole.forward(db)):
        assert torch.equal(a, b)
