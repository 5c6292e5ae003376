"""Several consecutive training steps against the FP64 oracle (Adam's bias corrections at step
counts 2 and 3, moments carried over).

Two comparisons per workload and precision:

* per step, from a common state: before step s both sides are given the oracle's state after
  step s - 1, rounded to FP32 (parameters, Adam moments, step count; pushed into the library
  with set_state), so every step is checked at the single-step tolerance on identical inputs;
* free running: the library and the oracle each take three steps from the initialisation on
  their own; the drift between the trajectories is reported (FP32 rounding compounds through
  Adam's sign-like early updates, so no tolerance of one step applies to it).
"""
import numpy as np
import pytest

import oracle
import scenes
from vmap_testlib import check_step, make_pair, relerr, report, scaled, step_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts, never run there
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2302_01838_amd as vm  # noqa: E402

STEPS = 3


def _scene(name):
    sc = scenes.make_scene("tiny_k4" if name == "tiny_k4" else "k50_uneven")
    return sc if name == "tiny_k4" else scaled(sc, 10)


def _sync(objs, states):
    """Round the oracle's states to FP32 and give the same values to both sides."""
    for k, st in states.items():
        th, m, v = (x.astype(np.float32) for x in (st.theta, st.m, st.v))
        objs.set_state(k, vm.STATE_PARAMS, th)
        objs.set_state(k, vm.STATE_ADAM_M, m)
        objs.set_state(k, vm.STATE_ADAM_V, v)
        objs.set_state(k, vm.STATE_STEP, st.t)
        st.theta, st.m, st.v = (x.astype(np.float64) for x in (th, m, v))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("name", ["tiny_k4", "k50_div10"])
def test_three_steps_from_common_states(name, precision):
    sc = _scene(name)
    objs, states = make_pair(sc, precision)
    for s in range(STEPS):
        _sync(objs, states)
        batch = scenes.make_batch(sc, s)
        errs, errs16, unstable, after = step_errors(objs, states, batch, precision, sc.B)
        report(f"multistep {name} {precision} step {s + 1} (sign-unstable={unstable})", **errs)
        if errs16:
            report(f"multistep {name} {precision} step {s + 1} vs bf16 oracle", **errs16)
        check_step(errs, errs16, precision)
        for k in states:
            assert objs.get_state(k, vm.STATE_STEP) == s + 1
        states = after


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_free_running_trajectory(precision):
    sc = _scene("tiny_k4")
    objs, states = make_pair(sc, precision)
    for s in range(STEPS):
        batch = scenes.make_batch(sc, s)
        loss = objs.step(vm.DeviceBatch(batch)).cpu().numpy()
        torch.cuda.synchronize()
        l_ref, _, _ = oracle.step(states, batch, sc.B)
        th = max(relerr(objs.get_state(k, vm.STATE_PARAMS), states[k].theta) for k in states)
        m = max(relerr(objs.get_state(k, vm.STATE_ADAM_M), states[k].m) for k in states)
        report(f"free-running {precision} step {s + 1}", loss=relerr(loss, l_ref), theta=th, m=m)
        # a loose sanity bound: the trajectories stay together to well within the updates' size
        assert relerr(loss, l_ref) <= 2e-2 and th <= 2e-2
