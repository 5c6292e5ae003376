"""The training step with its work list built inside the tile kernel, against the same step
with a separate work-list launch, through the C ABI.

By default a training step whose objects all have width 32 has every workgroup of the tile
kernel scan the batch's ray offsets into a tile table in LDS; workgroup 0 leaves the table, the
Adam step counts and cleared flags for the optimiser kernel, and tiles report non-finite partials
per tile. With ``split_step`` a work-list kernel does that first. Both sum the same partials in
the same order, so every result must agree bitwise: losses, parameters, Adam moments,
gradients, step counts and the scaler state. Parity with the FP64 oracle is covered by the parity
tests (which run the default form).
"""
import numpy as np
import pytest

import scenes
from vmap_testlib import make_pair, remap_batch, scaled

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, never run there
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2302_01838_amd as vm  # noqa: E402

WHAT = (vm.STATE_PARAMS, vm.STATE_ADAM_M, vm.STATE_ADAM_V, vm.STATE_GRAD)


def _assert_same(a, b, ids):
    for k in ids:
        for w in WHAT:
            x, y = a.get_state(k, w), b.get_state(k, w)
            assert np.array_equal(x, y, equal_nan=True), (k, w)
        assert a.get_state(k, vm.STATE_STEP) == b.get_state(k, vm.STATE_STEP), k
    assert a.step_info() == b.step_info()


def _pair(sc, precision, **kw):
    table, _ = make_pair(sc, precision, **kw)
    split, _ = make_pair(sc, precision, split_step=True, **kw)
    return table, split


def _run(table, split, batches):
    for i, batch in enumerate(batches):
        db = vm.DeviceBatch(batch)
        l1 = table.step(db).cpu().numpy()
        l2 = split.step(db).cpu().numpy()
        torch.cuda.synchronize()
        print(f"[table] step {i}: objects {len(batch['object_ids'])}, loss sum {np.nansum(l1):.6g}",
              flush=True)
        assert np.array_equal(l1, l2, equal_nan=True), i


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_table_step_matches_split_launches(precision):
    sc = scaled(scenes.make_scene("k50_uneven"), 10)
    table, split = _pair(sc, precision)
    # three steps; the second pauses two objects (zero rays) and the third drops one
    n = sc.n_objects
    batches = [scenes.make_batch(sc, 0),
               scenes.make_batch(sc, 1, n_rays={3: 0, 17: 0}),
               scenes.make_batch(sc, 2, object_ids=[k for k in range(n) if k != 5])]
    _run(table, split, batches)
    _assert_same(table, split, range(n))
    assert table.get_state(3, vm.STATE_STEP) == 2 and table.get_state(5, vm.STATE_STEP) == 2
    assert table.get_state(0, vm.STATE_STEP) == 3


@pytest.mark.parametrize("precision,rpt,waves,grid", [
    ("fp32", 1, 4, 0), ("bf16", 5, 2, 0), ("bf16", 0, 3, 0), ("fp32", 0, 1, 3), ("bf16", 0, 4, 7),
    ("bf16", 72, 8, 0), ("bf16", 0, 6, 5)])
def test_table_step_launch_shapes(precision, rpt, waves, grid):
    """One-ray tiles, one- to eight-wave workgroups (the table scan's wave count and the number of
    gradient copies differ) and grids smaller than the tile count (workgroups loop over tiles of
    several objects)."""
    sc = scaled(scenes.make_scene("k50_uneven"), 10)
    table, split = _pair(sc, precision, rays_per_tile=rpt)
    for o in (table, split):
        o.set_launch(waves, grid)
    _run(table, split, [scenes.make_batch(sc, s) for s in range(2)])
    _assert_same(table, split, range(sc.n_objects))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_table_step_without_rays(precision):
    """A batch whose objects all have zero rays updates nothing; the scaler still counts a good
    step."""
    sc = scenes.make_scene("tiny_k4")
    table, split = _pair(sc, precision)
    zero = scenes.make_batch(sc, 0, n_rays={k: 0 for k in range(4)})
    _run(table, split, [zero, scenes.make_batch(sc, 1), zero])
    _assert_same(table, split, range(4))
    assert table.get_state(0, vm.STATE_STEP) == 1


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_table_step_nonfinite_partial_skips_object(precision):
    """An infinite ray origin makes the encoding, and so the object's tile partial, NaN: that
    object keeps its parameters and step count, the others train, the skip is counted and (BF16)
    the loss scale halves."""
    sc = scaled(scenes.make_scene("k50_uneven"), 10)
    table, split = _pair(sc, precision)
    bad = scenes.make_batch(sc, 0)
    r = int(bad["ray_offsets"][4])  # first ray of object 4
    bad["rays_o"] = bad["rays_o"].copy()
    bad["rays_o"][r] = np.inf
    before = table.get_state(4, vm.STATE_PARAMS)
    scale0 = table.step_info()[0]
    _run(table, split, [bad])
    _assert_same(table, split, range(sc.n_objects))
    scale, skipped, err = table.step_info()
    assert skipped == 1 and err == 0
    assert scale == (scale0 / 2 if precision == "bf16" else 1.0)
    assert np.array_equal(table.get_state(4, vm.STATE_PARAMS), before)
    assert table.get_state(4, vm.STATE_STEP) == 0 and table.get_state(0, vm.STATE_STEP) == 1
    _run(table, split, [scenes.make_batch(sc, 1)])
    _assert_same(table, split, range(sc.n_objects))
    assert table.get_state(4, vm.STATE_STEP) == 1 and table.step_info()[1] == 0


def test_table_step_invalid_id():
    """An id beyond the stack raises the device flag; the valid objects still train."""
    sc = scenes.make_scene("tiny_k4")
    table, split = _pair(sc, "fp32", ids=[0, 1])
    batch = remap_batch(scenes.make_batch(sc, 0, object_ids=[0, 1]), [0, 1])
    batch["object_ids"] = np.asarray([0, 7], dtype=np.int32)
    _run(table, split, [batch])
    _assert_same(table, split, [0, 1])
    assert table.step_info()[2] == 1
    assert table.get_state(0, vm.STATE_STEP) == 1 and table.get_state(1, vm.STATE_STEP) == 0


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_table_step_graph_replay(precision):
    """Captured once, replayed over batches in different buffers, equal to plain split steps."""
    sc = scaled(scenes.make_scene("k50_uneven"), 10)
    table, split = _pair(sc, precision)
    table.set_graph_mode(True)
    _run(table, split, [scenes.make_batch(sc, s) for s in range(4)])
    _assert_same(table, split, range(sc.n_objects))


def test_table_step_at_table_capacity():
    """2048 batch objects (the LDS tile table's capacity) of one to three rays, two steps,
    against split launches."""
    n = 2048
    sc = scenes.make_scene("tiny_k4")
    pool = scenes.make_batch(sc, 0, object_ids=[0], n_rays={0: 3 * n})
    counts = 1 + (np.arange(n) * 7919) % 3
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    R = int(offs[-1])
    batch = {k: pool[k][:R] for k in ("rays_o", "rays_d", "t", "depth", "rgb", "mask")}
    batch.update(object_ids=np.arange(n, dtype=np.int32), ray_offsets=offs, S=pool["S"])
    sets = []
    for split_step in (False, True):
        o = vm.ObjectSet(max_objects=n, B=sc.B, precision="bf16", max_rays=R + 64,
                         max_samples_per_ray=sc.S, split_step=split_step)
        ob = sc.objects[0]
        for k in range(n):
            assert o.add(ob.norm_centre, ob.norm_scale, seed=1000 + k) == k
        sets.append(o)
    _run(sets[0], sets[1], [batch, batch])
    _assert_same(sets[0], sets[1], range(0, n, 97))
    for k in (0, n - 1):
        assert sets[0].get_state(k, vm.STATE_STEP) == 2
