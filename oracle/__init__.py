"""FP64 CPU oracle of the vectorised per-object training step (vMAP, arXiv 2302.01838).

TEST INFRASTRUCTURE ONLY. This package is the slow, plain reference that the GPU path is checked
against. Only the tests, the package entry's smoke check and the benchmark's CPU-baseline leg may
import it; the product path never does. It shares no code with the HIP library: the only common
module is ``scenes`` (seeded inputs, none of the step's arithmetic).

Everything here is float64 numpy written from the paper's definitions, in the paper's order and
notation, with numpy matmul as the only library primitive:

* point normalisation into the object's unit box (supplement Sec. B, object-level positional
  encoding: every object is scaled into [-1, 1]^3 by its own bound);
* Gaussian Fourier features gamma(x) = [sin(x B), cos(x B)] (the build's stand-in for the
  paper's integrated positional encoding, supplement Sec. B);
* one MLP per object: hidden ReLU layers and a linear head to (r, g, b, occupancy), with a
  sigmoid on every output (Sec. 3.3, "Surface and Volume Rendering": occupancy in [0, 1]);
* occupancy rendering, Eq. 3: T_i = o_i prod_{j<i}(1 - o_j); O = sum T_i, D = sum T_i t_i,
  C = sum T_i c_i;
* the per-object depth, colour and occupancy L1 losses (Eqs. 4-6) and the weighted total
  (Eq. 7, lambda_1 = 5, lambda_2 = 10);
* the gradient by plain reverse-mode differentiation of those steps;
* one Adam update per object (the optimiser is not named in the paper; Adam with lr 1e-3 is
  the workload's choice), skipped for objects without rays (Sec. 3.2: each object can be
  stopped or resumed without interfering with the others).

Readings where the paper is silent or garbled:

* losses are sums over the object's rays (Eqs. 4-6 as printed), the mask applies per ray, and
  the colour residual is the L1 norm over the three channels;
* B has entries of variance 25; phi = x B with no 2 pi factor; gamma lists all sines, then all
  cosines;
* depth d_i in Eq. 3 is the ray parameter t_i (unit directions);
* for a ray inside the mask the occupancy residual O - 1 is evaluated as -prod_i(1 - o_i),
  which equals it exactly and keeps its sign when O rounds to 1;
* sgn(0) = 0 for the L1 subgradient and ReLU'(0) = 0;
* Adam: beta = (0.9, 0.999), eps = 1e-8 added outside the square root, bias-corrected with
  each object's own step count, no weight decay;
* weights are Xavier-uniform with bound sqrt(6 / (fan_in + fan_out)), biases zero, the
  uniforms drawn from SplitMix64 (Steele, Lea and Flood 2014) in counter mode.

Parity is pinned in ``tests/test_oracle_pins.py`` by closed forms, brute force, finite
differences, torch's autograd and torch's Adam, and invariants. The absolute loss values of a
full step are pinned only by that composition: the paper prints no worked example.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import numpy as np

__all__ = [
    "LAMBDA_COLOUR", "LAMBDA_OCC", "N_OUT", "layer_shapes", "n_params", "unpack",
    "splitmix64", "xavier_init", "normalise", "encode", "mlp_forward", "heads", "render",
    "render_vjp", "ray_losses", "object_forward", "object_loss_and_grad", "adam_update",
    "ObjectState", "step", "query", "bf16_round", "splitmix64_array", "depth_guided_samples",
    "ray_box", "render_scene", "mlp_backward",
]

LAMBDA_COLOUR = 5.0   # lambda_1 of Eq. 7
LAMBDA_OCC = 10.0     # lambda_2 of Eq. 7
N_OUT = 4             # (r, g, b, occupancy)


# --------------------------------------------------------------------------- parameter layout

def layer_shapes(H: int, L: int, E: int) -> List[tuple]:
    """(fan_out, fan_in) of each linear map: E -> H (L times H -> H in total) -> 4."""
    widths = [E] + [H] * L + [N_OUT]
    return [(widths[i + 1], widths[i]) for i in range(len(widths) - 1)]


def n_params(H: int, L: int, E: int) -> int:
    return sum(o * i + o for o, i in layer_shapes(H, L, E))


def unpack(theta: np.ndarray, H: int, L: int, E: int):
    """Views (W_l [out, in], b_l [out]) into a flat parameter vector, in layout order."""
    out, off = [], 0
    for o, i in layer_shapes(H, L, E):
        W = theta[off:off + o * i].reshape(o, i)
        off += o * i
        b = theta[off:off + o]
        off += o
        out.append((W, b))
    assert off == theta.shape[0]
    return out


# --------------------------------------------------------------------------- initialisation

_MASK64 = (1 << 64) - 1


def splitmix64(seed: int, index: np.ndarray) -> np.ndarray:
    """Output number ``index`` (0-based) of a SplitMix64 stream started at state ``seed``.

    The state advances by the odd constant 0x9E3779B97F4A7C15 and every output is the state's
    avalanche mix (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
    OOPSLA 2014). Evaluated in Python integers so the wrap-around is explicit.
    """
    out = np.empty(len(index), dtype=np.uint64)
    for j, n in enumerate(np.asarray(index, dtype=np.int64).tolist()):
        z = (int(seed) + (n + 1) * 0x9E3779B97F4A7C15) & _MASK64
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        out[j] = z ^ (z >> 31)
    return out


def splitmix64_array(seed: int, index: np.ndarray) -> np.ndarray:
    """``splitmix64`` for many indices at once, in numpy uint64 (arithmetic modulo 2^64)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.asarray(index, dtype=np.uint64) + np.uint64(1)) * \
            np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def xavier_init(seed: int, H: int, L: int, E: int) -> np.ndarray:
    """Xavier-uniform weights, zero biases, as the FP32 vector both sides start from.

    Parameter p of the flat layout draws u_p = (top 24 bits of output p) * 2^-24 in [0, 1);
    a weight of a layer with bound a = sqrt(6 / (fan_in + fan_out)) is a * (2 u_p - 1),
    evaluated in FP64 and rounded once to FP32.
    """
    P = n_params(H, L, E)
    bits = splitmix64(seed, np.arange(P))
    u = (bits >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    theta = np.zeros(P, dtype=np.float64)
    off = 0
    for o, i in layer_shapes(H, L, E):
        a = np.sqrt(6.0 / (i + o))
        theta[off:off + o * i] = a * (2.0 * u[off:off + o * i] - 1.0)
        off += o * i + o
    return theta.astype(np.float32)


# --------------------------------------------------------------------------- BF16 diagnosis

def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), via FP32, returned as FP64.

    BF16 keeps the upper 16 bits of an IEEE binary32 value. Round to nearest, ties to even, adds
    0x7FFF plus the lowest kept bit to the pattern and drops the lower half; a finite value whose
    magnitude rounds past the largest BF16 value becomes an infinity of its sign. NaN stays NaN
    (the carry would otherwise turn a small payload into an infinity or wrap the pattern).

    Only for the optional BF16 diagnostic modes: they tell the error that BF16 products bring by
    themselves apart from the GPU's accumulation order. The default mode is pure FP64.
    """
    f = np.asarray(x, dtype=np.float32)
    u = np.ascontiguousarray(f).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    with np.errstate(invalid="ignore"):  # NaN patterns, replaced below
        out = u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(f.shape)
    return np.where(np.isnan(f), np.nan, out)


def _identity(x):
    return x


# --------------------------------------------------------------------------- forward pieces

def normalise(rays_o, rays_d, t, centre, scale) -> np.ndarray:
    """x = (o + t d - c) / s for every sample: [R, S, 3] in FP64."""
    o = np.asarray(rays_o, np.float64)[:, None, :]
    d = np.asarray(rays_d, np.float64)[:, None, :]
    tt = np.asarray(t, np.float64)[:, :, None]
    c = np.asarray(centre, np.float64)
    return (o + tt * d - c) / np.float64(scale)


def encode(x: np.ndarray, B: np.ndarray, var: Optional[np.ndarray] = None) -> np.ndarray:
    """gamma = [sin(x B), cos(x B)] over the last axis (3 -> 2F).

    With ``var`` (one variance per point, same leading shape as x) the point stands for an
    isotropic Gaussian N(x, var I) and each feature becomes its expectation under it, the
    integrated positional encoding of the supplement's object-level encoding (after mip-NeRF
    360): E[sin(x' b)] = sin(x b) exp(-var |b|^2 / 2), likewise for the cosine, b a column of B.
    """
    B = np.asarray(B, np.float64)
    phi = x @ B
    if var is None:
        return np.concatenate([np.sin(phi), np.cos(phi)], axis=-1)
    att = np.exp(-0.5 * np.asarray(var, np.float64)[..., None] * np.sum(B * B, axis=0))
    return np.concatenate([np.sin(phi) * att, np.cos(phi) * att], axis=-1)


def mlp_forward(theta: np.ndarray, gamma: np.ndarray, H: int, L: int, rnd=_identity,
                relu_masks=None):
    """Rows of ``gamma`` through the object's MLP. Returns z [N, 4] and the pre-activations.

    ``rnd`` is applied to both operands of every product (identity: exact FP64; bf16_round:
    the diagnostic BF16 mode). ``relu_masks`` (one boolean [N, H] per hidden layer) replaces the
    ReLU's own decision a > 0 by a given one: h = a where the mask is set, else 0.
    """
    layers = unpack(np.asarray(theta, np.float64), H, L, gamma.shape[-1])
    h = gamma
    pre = []
    for li, (W, b) in enumerate(layers[:-1]):
        a = rnd(h) @ rnd(W).T + b
        pre.append(a)
        h = np.maximum(a, 0.0) if relu_masks is None else np.where(relu_masks[li], a, 0.0)
    W, b = layers[-1]
    return rnd(h) @ rnd(W).T + b, pre


def _sigmoid(z):
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-z))


def heads(z: np.ndarray):
    """c = sigmoid(z[..., :3]) (colour), o = sigmoid(z[..., 3]) (occupancy)."""
    return _sigmoid(z[..., :3]), _sigmoid(z[..., 3])


def render(o: np.ndarray, c: np.ndarray, t: np.ndarray):
    """Eq. 3 along each ray. o, t [R, S]; c [R, S, 3].

    Returns (O_hat [R], D_hat [R], C_hat [R, 3], T [R, S], P [R, S+1]) where P_i is the
    product of (1 - o_j) over the samples before i, so T_i = o_i P_i and P_{S+1} is what is
    left after the last sample.
    """
    R, S = o.shape
    P = np.empty((R, S + 1))
    P[:, 0] = 1.0
    for i in range(S):
        P[:, i + 1] = P[:, i] * (1.0 - o[:, i])
    T = o * P[:, :S]
    return T.sum(1), (T * t).sum(1), (T[:, :, None] * c).sum(1), T, P


def render_vjp(o, c, t, gO, gD, gC, gPend):
    """Reverse-mode derivative of ``render``: cotangents of (O, D, C, P_{S+1}) -> (do, dc).

    Walks the recurrence P_{i+1} = P_i (1 - o_i) backwards from the last sample.
    """
    R, S = o.shape
    _, _, _, T, P = render(o, c, t)
    gT = gO[:, None] + gD[:, None] * t + np.einsum("rk,rsk->rs", gC, c)
    do = np.zeros((R, S))
    gP_next = np.asarray(gPend, np.float64).copy()      # cotangent of P_{i+1}
    for i in range(S - 1, -1, -1):
        # T_i = o_i P_i and P_{i+1} = P_i (1 - o_i)
        do[:, i] = gT[:, i] * P[:, i] - gP_next * P[:, i]
        gP_next = gT[:, i] * o[:, i] + gP_next * (1.0 - o[:, i])
    dc = T[:, :, None] * gC[:, None, :]
    return do, dc


def _sgn(x):
    return np.sign(x)   # sign(0) = 0


def ray_losses(O, D, C, P_end, depth, rgb, mask):
    """Per-ray terms of Eqs. 4-6 and the occupancy residual rho.

    rho = O - M, computed as -P_{S+1} where M = 1 (exactly equal, see module notes).
    """
    rho = np.where(mask == 1.0, -P_end, O - mask)
    l_depth = mask * np.abs(D - depth)
    l_colour = mask * np.abs(C - rgb).sum(-1)
    l_occ = np.abs(rho)
    return l_depth, l_colour, l_occ, rho


# --------------------------------------------------------------------------- one object

def object_forward(theta, H, L, B, centre, scale, rays_o, rays_d, t, rnd=_identity, var=None,
                   relu_masks=None):
    """Encode + MLP + heads + render for one object's rays. Returns a dict of intermediates.

    ``var`` [R, S]: per-sample variance of the sample's Gaussian in world units squared (the
    integrated encoding), or None for point samples; the object frame divides it by s^2.
    ``relu_masks``: given ReLU decisions (see ``mlp_forward``); ``masks`` in the result holds the
    decisions used.
    """
    R, S = np.shape(t)
    x = normalise(rays_o, rays_d, t, centre, scale)
    vn = None if var is None else np.asarray(var, np.float64) / np.float64(scale) ** 2
    gamma = encode(x, B, vn)
    z, pre = mlp_forward(theta, gamma.reshape(R * S, -1), H, L, rnd, relu_masks)
    masks = [a > 0.0 for a in pre] if relu_masks is None else list(relu_masks)
    c, o = heads(z)
    c = c.reshape(R, S, 3)
    o = o.reshape(R, S)
    tt = np.asarray(t, np.float64)
    O, D, C, T, P = render(o, c, tt)
    return dict(x=x, gamma=gamma.reshape(R * S, -1), pre=pre, masks=masks, z=z, c=c, o=o, t=tt,
                O=O, D=D, C=C, T=T, P=P)


def object_loss_and_grad(theta, H, L, B, centre, scale, rays_o, rays_d, t, depth, rgb, mask,
                         upstream: float = 1.0, want_grad: bool = True, rnd=_identity, var=None,
                         decide=None):
    """L^k of Eq. 7 for one object and, optionally, upstream * dL^k/dtheta.

    Returns (loss, grad or None, forward dict). With ``rnd`` = bf16_round every product of the
    MLP (forward and backward, the output layer's seed dz included) takes BF16-rounded operands;
    bias gradients sum the rounded deltas, except the output layer's, which sums dz itself
    (diagnostic mode).

    ``decide`` (a rounding function, e.g. bf16_round) takes the step's integer decisions -- each
    ReLU's a > 0 and the sign of each L1 residual -- in a forward pass whose products round their
    operands with it, and the arithmetic (``rnd``) then follows those decisions: the gradient of
    the piece of the piecewise-smooth loss that the lower-precision forward selects, evaluated in
    the precision of ``rnd``.
    """
    depth = np.asarray(depth, np.float64)
    rgb = np.asarray(rgb, np.float64)
    mask = np.asarray(mask, np.float64)
    relu_masks = None
    if decide is not None:
        fd = object_forward(theta, H, L, B, centre, scale, rays_o, rays_d, t, decide, var)
        relu_masks = fd["masks"]
    fw = object_forward(theta, H, L, B, centre, scale, rays_o, rays_d, t, rnd, var, relu_masks)
    R, S = fw["o"].shape
    ld, lc, lo, rho = ray_losses(fw["O"], fw["D"], fw["C"], fw["P"][:, S], depth, rgb, mask)
    loss = float(np.sum(ld) + LAMBDA_COLOUR * np.sum(lc) + LAMBDA_OCC * np.sum(lo))
    if not want_grad:
        return loss, None, fw
    theta64 = np.asarray(theta, np.float64)
    # signs of the residuals (L1 subgradients), from the deciding forward if there is one
    sD, sC, s_rho = _sgn(fw["D"] - depth), _sgn(fw["C"] - rgb), _sgn(rho)
    if decide is not None:
        _, _, _, rho_d = ray_losses(fd["O"], fd["D"], fd["C"], fd["P"][:, S], depth, rgb, mask)
        sD, sC, s_rho = _sgn(fd["D"] - depth), _sgn(fd["C"] - rgb), _sgn(rho_d)
    # cotangents of the rendered quantities
    gD = upstream * mask * sD
    gC = upstream * LAMBDA_COLOUR * mask[:, None] * sC
    g_rho = upstream * LAMBDA_OCC * s_rho
    inside = mask == 1.0
    gO = np.where(inside, 0.0, g_rho)           # rho = O - M when M = 0
    gPend = np.where(inside, -g_rho, 0.0)       # rho = -P_{S+1} when M = 1
    do, dc = render_vjp(fw["o"], fw["c"], fw["t"], gO, gD, gC, gPend)
    # through the sigmoids to the head outputs
    dz = np.empty((R * S, N_OUT))
    cf = fw["c"].reshape(R * S, 3)
    of = fw["o"].reshape(R * S)
    dz[:, :3] = dc.reshape(R * S, 3) * cf * (1.0 - cf)
    dz[:, 3] = do.reshape(R * S) * of * (1.0 - of)
    g = mlp_backward(theta64, H, L, fw["gamma"], fw["pre"], fw["masks"], dz, rnd)
    return loss, g, fw


def mlp_backward(theta, H: int, L: int, gamma, pre, masks, dz, rnd=_identity):
    """Reverse mode through the MLP, last layer first: the flat gradient for the seed dz [N, 4].

    delta_out = dz; dW_l = delta_l^T h_{l-1}, db_l = sum over rows of delta_l; delta_{l-1} =
    (delta_l W_l) * ReLU'(a_{l-1}), with ReLU' the forward's decision ``masks``. ``rnd`` rounds
    both operands of every product; bias gradients sum the deltas as the products see them,
    except at the output layer, whose seed dz is summed unrounded.
    """
    layers = unpack(np.asarray(theta, np.float64), H, L, gamma.shape[-1])
    hs = [gamma] + [np.where(m, a, 0.0) for a, m in zip(pre, masks)]
    grads = []
    delta = dz
    last = len(layers) - 1
    for li in range(last, -1, -1):
        W, _ = layers[li]
        d_op = rnd(delta)
        grads.append((d_op.T @ rnd(hs[li]), (delta if li == last else d_op).sum(0)))
        if li > 0:
            delta = (d_op @ rnd(W)) * masks[li - 1]
    grads.reverse()
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def adam_update(theta, m, v, g, step_count, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step with bias correction at step ``step_count`` (already incremented)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step_count)
    v_hat = v / (1.0 - beta2 ** step_count)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


# --------------------------------------------------------------------------- sampling

def depth_guided_samples(t_near, t_far, depth, S: int, n_strat: int, sigma: float, seed: int):
    """Depth-guided samples of Sec. 3.3 (Eqs. 1 and 2), sorted per ray: [R, S] FP64.

    t_s is the observed depth where it is valid (> 0) and the far bound otherwise. Sample i < N_c
    is stratified: t_n + (i + u) / N_c * (t_s - t_n); the others are t_s + sigma * z with z
    standard normal (Box-Muller: z = sqrt(-2 ln u1) cos(2 pi u2)). Uniform j of sample i of ray r
    comes from output 2 (r S + i) + j of the SplitMix64 stream started at ``seed``:
    u = top 24 bits * 2^-24, and u1 = (top 24 bits + 1) * 2^-24 so that ln u1 is finite.
    """
    t_near = np.asarray(t_near, np.float64)
    t_far = np.asarray(t_far, np.float64)
    depth = np.asarray(depth, np.float64)
    R = t_near.shape[0]
    t_s = np.where(depth > 0.0, depth, t_far)
    idx = (np.arange(R)[:, None] * S + np.arange(S)[None, :]).astype(np.uint64) * np.uint64(2)
    top0 = (splitmix64_array(seed, idx) >> np.uint64(40)).astype(np.float64)
    top1 = (splitmix64_array(seed, idx + np.uint64(1)) >> np.uint64(40)).astype(np.float64)
    i = np.arange(S)[None, :]
    strat = t_near[:, None] + (i + top0 * 2.0 ** -24) / n_strat * (t_s - t_near)[:, None]
    z = np.sqrt(-2.0 * np.log((top0 + 1.0) * 2.0 ** -24)) * np.cos(2.0 * np.pi * top1 * 2.0 ** -24)
    near = t_s[:, None] + sigma * z
    t = np.where(i < n_strat, strat, near)
    return np.sort(t, axis=1)


# --------------------------------------------------------------------------- the step

class ObjectState:
    """Parameters, Adam moments and step count of one object model, all FP64."""

    def __init__(self, theta, H: int, L: int, centre, scale):
        self.theta = np.asarray(theta, np.float64).copy()
        self.m = np.zeros_like(self.theta)
        self.v = np.zeros_like(self.theta)
        self.t = 0
        self.H, self.L = int(H), int(L)
        self.centre = np.asarray(centre, np.float64)
        self.scale = float(scale)

    def copy(self) -> "ObjectState":
        c = ObjectState(self.theta, self.H, self.L, self.centre, self.scale)
        c.m, c.v, c.t = self.m.copy(), self.v.copy(), self.t
        return c


def step(states: Dict[int, ObjectState], batch: dict, B, lr=1e-3, beta1=0.9, beta2=0.999,
         eps=1e-8, apply_adam: bool = True, upstream: Optional[Sequence[float]] = None,
         rnd=_identity, decide=None):
    """One training step over a CSR batch; objects are independent and processed in order.

    Returns (losses [n] FP64, grads {id: g}, renders dict with O, D, C per ray). ``states`` is
    updated in place when ``apply_adam`` is true; objects with no rays are left untouched.
    ``rnd`` and ``decide`` as in ``object_loss_and_grad``.
    """
    ids = [int(k) for k in batch["object_ids"]]
    offs = np.asarray(batch["ray_offsets"], np.int64)
    R = int(offs[-1])
    var = batch.get("var")
    losses = np.zeros(len(ids))
    grads = {}
    O = np.zeros(R)
    D = np.zeros(R)
    C = np.zeros((R, 3))
    for j, k in enumerate(ids):
        r0, r1 = offs[j], offs[j + 1]
        st = states[k]
        if r1 == r0:
            grads[k] = np.zeros_like(st.theta)
            continue
        up = 1.0 if upstream is None else float(upstream[j])
        loss, g, fw = object_loss_and_grad(
            st.theta, st.H, st.L, B, st.centre, st.scale, batch["rays_o"][r0:r1],
            batch["rays_d"][r0:r1], batch["t"][r0:r1], batch["depth"][r0:r1],
            batch["rgb"][r0:r1], batch["mask"][r0:r1], upstream=up, rnd=rnd, decide=decide,
            var=None if var is None else var[r0:r1])
        losses[j] = loss
        grads[k] = g
        O[r0:r1], D[r0:r1], C[r0:r1] = fw["O"], fw["D"], fw["C"]
        if apply_adam:
            st.t += 1
            st.theta, st.m, st.v = adam_update(st.theta, st.m, st.v, g, st.t, lr, beta1, beta2,
                                               eps)
    return losses, grads, dict(O=O, D=D, C=C)


def query(theta, H: int, L: int, B, centre, scale, pts):
    """Occupancy and colour of world-frame points inside one object's bound."""
    x = (np.asarray(pts, np.float64) - np.asarray(centre, np.float64)) / np.float64(scale)
    z, _ = mlp_forward(theta, encode(x, B), H, L)
    c, o = heads(z)
    return o, c


# --------------------------------------------------------------------------- scene rendering

def ray_box(rays_o, rays_d, lo, hi):
    """Entry and exit parameters (t0, t1) of each ray against the axis-aligned box [lo, hi]:
    the slab method (Kay and Kajiya 1986), the ray-box intersection Sec. 3.4 relies on. Per
    axis the ray is inside the slab for t between (lo - o)/d and (hi - o)/d (in either order);
    the box is the intersection of the three slabs. A direction component of zero leaves the
    ray inside that slab for all t when its origin lies within it, and never otherwise."""
    o = np.asarray(rays_o, np.float64)
    d = np.asarray(rays_d, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    t0 = np.full(o.shape[0], -np.inf)
    t1 = np.full(o.shape[0], np.inf)
    for a in range(3):
        par = d[:, a] == 0.0
        inside = (o[:, a] >= lo[a]) & (o[:, a] <= hi[a])
        with np.errstate(divide="ignore", invalid="ignore"):
            ta = (lo[a] - o[:, a]) / d[:, a]
            tb = (hi[a] - o[:, a]) / d[:, a]
        near = np.where(par, np.where(inside, -np.inf, np.inf), np.minimum(ta, tb))
        far = np.where(par, np.where(inside, np.inf, -np.inf), np.maximum(ta, tb))
        t0 = np.maximum(t0, near)
        t1 = np.minimum(t1, far)
    return t0, t1


def render_scene(states: Sequence[ObjectState], B, rays_o, rays_d, S: int, t_min: float = 0.0,
                 occ_threshold: float = 0.5, per_object: Optional[list] = None):
    """Occlusion-aware rendering of a scene recomposed from object models (Sec. 3.4).

    For every object, the rays that meet its bound [c - s, c + s]^3 (``ray_box``) are sampled at
    the midpoints of S equal parts of [max(t0, t_min), t1] (rounded to FP32, the precision of
    the sample depths the step consumes) and rendered with the object's own MLP (Eq. 3). Each ray
    then ranks the objects it met by rendered depth and takes the nearest one whose rendered
    occupancy reaches ``occ_threshold`` (an equal depth keeps the lower object index).

    Returns depth [R], rgb [R, 3], occupancy [R] and object index [R] (-1 where no object
    qualifies; depth, rgb and occupancy are 0 there). If ``per_object`` is a list, each object's
    (ray indices, O, D, C) is appended to it.
    """
    R = np.shape(rays_o)[0]
    best_d = np.full(R, np.inf)
    out_c = np.zeros((R, 3))
    out_o = np.zeros(R)
    out_k = np.full(R, -1, dtype=np.int64)
    for k, st in enumerate(states):
        c = np.asarray(st.centre, np.float64)
        s = np.float64(st.scale)
        t0, t1 = ray_box(rays_o, rays_d, c - s, c + s)
        t0 = np.maximum(t0, t_min)
        hit = np.nonzero(t1 > t0)[0]
        if hit.size == 0:
            if per_object is not None:
                per_object.append((hit, np.zeros(0), np.zeros(0), np.zeros((0, 3))))
            continue
        frac = (np.arange(S, dtype=np.float64) + 0.5) / S
        t = t0[hit, None] + frac[None, :] * (t1[hit] - t0[hit])[:, None]
        t = t.astype(np.float32).astype(np.float64)
        fw = object_forward(st.theta, st.H, st.L, B, c, s, np.asarray(rays_o)[hit],
                            np.asarray(rays_d)[hit], t)
        if per_object is not None:
            per_object.append((hit, fw["O"], fw["D"], fw["C"]))
        take = (fw["O"] >= occ_threshold) & (fw["D"] < best_d[hit])
        r = hit[take]
        best_d[r] = fw["D"][take]
        out_c[r] = fw["C"][take]
        out_o[r] = fw["O"][take]
        out_k[r] = k
    depth = np.where(out_k >= 0, best_d, 0.0)
    return depth, out_c, out_o, out_k
