"""Planted mistakes in the oracle (on the CPU) must each fail at least one of its pins.

Every mutation below is a plausible slip when writing the oracle from the paper: a dropped term,
a wrong sign or index, a swapped head, a transposed operand. The test patches it into the oracle
module, runs the pins that should notice, and requires at least one of them to fail.
"""
import numpy as np
import pytest

import oracle
import test_oracle_bf16_pins as bf16_pins
import test_oracle_pins as pins


def _render_no_shift(o, c, t):
    # T_i uses the product up to and including sample i (index off by one)
    R, S = o.shape
    P = np.empty((R, S + 1))
    P[:, 0] = 1.0
    for i in range(S):
        P[:, i + 1] = P[:, i] * (1.0 - o[:, i])
    T = o * P[:, 1:]
    return T.sum(1), (T * t).sum(1), (T[:, :, None] * c).sum(1), T, P


_orig_render = oracle.render
_orig_vjp = oracle.render_vjp
_orig_heads = oracle.heads
_orig_mlp = oracle.mlp_forward
_orig_adam = oracle.adam_update
_orig_encode = oracle.encode
_orig_ray_losses = oracle.ray_losses
_orig_render_scene = oracle.render_scene
_orig_mlp_backward = oracle.mlp_backward


def _vjp_sign(o, c, t, gO, gD, gC, gPend):
    do, dc = _orig_vjp(o, c, t, gO, gD, gC, -np.asarray(gPend))
    return do, dc


def _heads_swapped(z):
    return _orig_heads(z[..., [3, 1, 2, 0]])


def _mlp_no_relu(theta, gamma, H, L, rnd=None, relu_masks=None):
    layers = oracle.unpack(np.asarray(theta, np.float64), H, L, gamma.shape[-1])
    h = gamma
    pre = []
    for W, b in layers[:-1]:
        a = h @ W.T + b
        pre.append(a)
        h = a
    W, b = layers[-1]
    return h @ W.T + b, pre


def _adam_no_bias_correction(theta, m, v, g, step_count, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    return theta - lr * m / (np.sqrt(v) + eps), m, v


def _encode_ipe_no_half(x, B, var=None):
    # the Gaussian's attenuation without the 1/2 of the exponent
    if var is None:
        return _orig_encode(x, B)
    return _orig_encode(x, B, 2.0 * np.asarray(var))


def _encode_swapped(x, B, var=None):
    phi = x @ np.asarray(B, np.float64)
    return np.concatenate([np.cos(phi), np.sin(phi)], axis=-1)


def _losses_no_colour_mask(O, D, C, P_end, depth, rgb, mask):
    ld, lc, lo, rho = _orig_ray_losses(O, D, C, P_end, depth, rgb, mask)
    return ld, np.abs(C - rgb).sum(-1), lo, rho


def _ray_box_union(rays_o, rays_d, lo, hi):
    # the union of the three slabs instead of their intersection
    o = np.asarray(rays_o, np.float64)
    d = np.asarray(rays_d, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        ta = (np.asarray(lo) - o) / d
        tb = (np.asarray(hi) - o) / d
    return np.nanmin(np.minimum(ta, tb), axis=1), np.nanmax(np.maximum(ta, tb), axis=1)


def _render_scene_no_threshold(*args, **kw):
    # every object met counts as seen, whatever its rendered occupancy
    kw["occ_threshold"] = -1.0
    return _orig_render_scene(*args, **kw)


def _bf16_truncate(x):
    # rounding toward zero (the lower 16 bits dropped) instead of to nearest even
    f = np.asarray(x, dtype=np.float32)
    u = np.ascontiguousarray(f).view(np.uint32) & np.uint32(0xFFFF0000)
    return u.view(np.float32).astype(np.float64).reshape(f.shape)


def _mlp_backward_seed_unrounded(theta, H, L, gamma, pre, masks, dz, rnd=None):
    # the output layer's seed dz enters its products unrounded
    rnd = rnd or (lambda x: x)
    layers = oracle.unpack(np.asarray(theta, np.float64), H, L, gamma.shape[-1])
    hs = [gamma] + [np.where(m, a, 0.0) for a, m in zip(pre, masks)]
    grads, delta, last = [], dz, len(layers) - 1
    for li in range(last, -1, -1):
        W, _ = layers[li]
        d_op = delta if li == last else rnd(delta)
        grads.append((d_op.T @ rnd(hs[li]), (delta if li == last else d_op).sum(0)))
        if li > 0:
            delta = (d_op @ rnd(W)) * masks[li - 1]
    grads.reverse()
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


MUTATIONS = {
    "render_index_off_by_one": ("render", _render_no_shift),
    "vjp_wrong_sign_of_leftover_transmittance": ("render_vjp", _vjp_sign),
    "occupancy_and_red_heads_swapped": ("heads", _heads_swapped),
    "relu_dropped": ("mlp_forward", _mlp_no_relu),
    "adam_without_bias_correction": ("adam_update", _adam_no_bias_correction),
    "sin_cos_swapped": ("encode", _encode_swapped),
    "integrated_encoding_without_half": ("encode", _encode_ipe_no_half),
    "colour_loss_not_masked": ("ray_losses", _losses_no_colour_mask),
    "ray_box_union_of_slabs": ("ray_box", _ray_box_union),
    "scene_ranking_ignores_occupancy": ("render_scene", _render_scene_no_threshold),
    "bf16_truncates_instead_of_nearest_even": ("bf16_round", _bf16_truncate),
    "bf16_output_seed_unrounded": ("mlp_backward", _mlp_backward_seed_unrounded),
}

PINS = [
    pins.test_encoding_at_origin,
    pins.test_mlp_forward_matches_torch_linear,
    pins.test_render_brute_force_product,
    pins.test_render_special_cases,
    pins.test_render_vjp_closed_form,
    pins.test_loss_hand_example,
    lambda: pins.test_render_constant_occupancy_closed_form(0.3, 10),
    lambda: pins.test_gradient_matches_torch_autograd(0),
    pins.test_adam_first_step_closed_form,
    pins.test_adam_second_step_values,
    pins.test_adam_matches_torch_optim,
    pins.test_ray_box_against_brute_force,
    pins.test_render_scene_ranks_constant_occupancy_objects,
    pins.test_integrated_encoding_is_the_gaussian_expectation,
    bf16_pins.test_bf16_round_matches_torch_cast,
    lambda: bf16_pins.test_bf16_mode_gradient_matches_torch_objective(0),
    lambda: bf16_pins.test_decided_gradient_matches_torch_with_fixed_pieces(0),
]


@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(oracle, attr, fn)
    failures = 0
    for pin in PINS:
        try:
            pin()
        except (AssertionError, ValueError, IndexError):
            failures += 1
    assert failures > 0, f"no pin caught the planted mistake {name}"
