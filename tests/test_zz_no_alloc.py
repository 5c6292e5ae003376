"""The allocation-free scene render (vmap_render_scene_static) against the render with a caller
scratch (vmap_render_scene), through the C ABI: two calls in a row, the second with fewer rays,
objects and samples, must give bitwise the same outputs; a scene too large for the static array
is refused before anything runs."""
import ctypes

import numpy as np
import pytest

import scenes
from vmap_testlib import make_pair, scaled

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, never run there
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2302_01838_amd as vm  # noqa: E402

VMAP_ECAPACITY = 2
STATIC_BYTES = 16 << 20  # VMAP_SCENE_STATIC_SCRATCH_BYTES


def _rays(sc, ids, n, seed):
    rng = np.random.default_rng(seed)
    o = rng.uniform(0.3, sc.room - 0.3, size=(n, 3))
    tgt = np.stack([sc.objects[int(k)].centre for k in rng.choice(ids, size=n)])
    tgt = tgt + rng.normal(0.0, 0.3, size=(n, 3))
    d = tgt - o
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    f = lambda x: torch.as_tensor(x.astype(np.float32)).cuda().contiguous()
    return f(o), f(d)


def _outputs(R):
    return (torch.full((R,), -7.0, device="cuda"), torch.full((R, 3), -7.0, device="cuda"),
            torch.full((R,), -7.0, device="cuda"), torch.full((R,), -9, dtype=torch.int32, device="cuda"),
            torch.full((1,), -9, dtype=torch.int32, device="cuda"))


def _call(objs, static, ro, rd, ids, S, max_pairs):
    lib = objs.lib
    R, n = ro.shape[0], ids.numel()
    out = _outputs(R)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    common = (objs.ctx, R, ro.data_ptr(), rd.data_ptr(), n, ids.data_ptr(), S, ctypes.c_float(0.0),
              ctypes.c_float(0.5), max_pairs)
    tail = tuple(t.data_ptr() for t in out) + (stream,)
    if static:
        rc = lib.vmap_render_scene_static(*common, *tail)
        keep = None
    else:
        nbytes = lib.vmap_scene_scratch_bytes(R, n, max_pairs, S)
        keep = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = (keep.data_ptr() + 255) // 256 * 256
        rc = lib.vmap_render_scene(*common, base, nbytes, *tail)
    torch.cuda.synchronize()
    return rc, [t.cpu().numpy() for t in out]


def test_static_scratch_scene_render_matches_caller_scratch():
    sc = scaled(scenes.make_scene("room50_background"), 8)
    ids = [50] + list(range(11))                       # background (hidden 128) + 11 objects
    objs, _ = make_pair(sc, "bf16", ids=ids, max_rays=20000)
    cases = [(3000, list(range(12)), 16, 20000),      # first call
             (700, [0, 3, 5, 6, 9], 8, 2000)]          # second call: smaller in every size
    for i, (R, lids, S, max_pairs) in enumerate(cases):
        ro, rd = _rays(sc, [ids[j] for j in lids], R, seed=11 + i)
        kid = torch.as_tensor(np.asarray(lids, np.int32)).cuda()
        print(f"[no-alloc] call {i}: rays {R}, objects {len(lids)}, S {S}, max_pairs {max_pairs}",
              flush=True)
        assert vm.load_library().vmap_scene_scratch_bytes(R, len(lids), max_pairs, S) <= STATIC_BYTES
        rc_s, got = _call(objs, True, ro, rd, kid, S, max_pairs)
        rc_c, want = _call(objs, False, ro, rd, kid, S, max_pairs)
        assert rc_s == 0 and rc_c == 0
        for g, w in zip(got, want):
            assert np.array_equal(g, w), i
        assert got[4][0] > 0 and np.any(got[3] >= 0)
    # too large for the static array (otherwise valid): refused before anything is enqueued,
    # outputs untouched
    big = vm.ObjectSet(max_objects=1, B=sc.B, precision="bf16", max_rays=65536,
                       max_samples_per_ray=64)
    ob = sc.objects[0]
    big.add(ob.norm_centre, ob.norm_scale, seed=ob.seed)
    R, S, max_pairs = 4000, 64, 65536
    assert vm.load_library().vmap_scene_scratch_bytes(R, 1, max_pairs, S) > STATIC_BYTES
    ro, rd = _rays(sc, [0], R, seed=3)
    kid = torch.zeros(1, dtype=torch.int32, device="cuda")
    rc, got = _call(big, True, ro, rd, kid, S, max_pairs)
    assert rc == VMAP_ECAPACITY
    assert b"static" in big.lib.vmap_last_error(big.ctx)
    assert np.all(got[0] == -7.0) and np.all(got[3] == -9)
    rc, got = _call(big, False, ro, rd, kid, S, max_pairs)  # the caller-scratch form takes it
    assert rc == 0 and got[4][0] > 0
