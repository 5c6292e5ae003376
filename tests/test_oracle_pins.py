"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against a closed form, a brute-force evaluation, central finite
differences, an independent library (torch autograd / torch.optim.Adam / torch.nn.Linear, all
float64 on the CPU), a published test vector, or an invariant of the method. Together they are
chosen so that a dropped term, a wrong sign or index, or a transposed operand in the oracle fails
at least one of them (see ``test_oracle_mutations.py``).
"""
import json
import math
import os

import numpy as np
import pytest
import torch
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- helpers

def tiny_problem(seed, R=3, S=4, H=4, L=2, F=3, margin=1e-3, max_tries=2000):
    """A small random object whose loss is smooth around theta (all kinks farther than margin)."""
    rng = np.random.default_rng(seed)
    for _ in range(max_tries):
        E = 2 * F
        P = oracle.n_params(H, L, E)
        theta = rng.normal(0.0, 0.7, size=P)
        B = rng.normal(0.0, 1.5, size=(3, F))
        centre = rng.normal(0.0, 0.3, size=3)
        scale = rng.uniform(0.5, 1.5)
        o = rng.normal(0.0, 1.0, size=(R, 3)) + np.array([0.0, 0.0, -3.0])
        d = rng.normal(0.0, 0.2, size=(R, 3)) + np.array([0.0, 0.0, 1.0])
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        t = np.sort(rng.uniform(2.0, 4.0, size=(R, S)), axis=1)
        depth = rng.uniform(2.0, 4.0, size=R)
        rgb = rng.uniform(0.0, 1.0, size=(R, 3))
        mask = (rng.uniform(size=R) < 0.6).astype(np.float64)
        fw = oracle.object_forward(theta, H, L, B, centre, scale, o, d, t)
        _, _, _, rho = oracle.ray_losses(fw["O"], fw["D"], fw["C"], fw["P"][:, S], depth, rgb,
                                         mask)
        ok = all(np.min(np.abs(a)) > margin for a in fw["pre"])
        ok &= np.min(np.abs(fw["D"] - depth)) > margin
        ok &= np.min(np.abs(fw["C"] - rgb)) > margin
        ok &= np.min(np.abs(rho)) > margin
        if ok:
            return dict(theta=theta, H=H, L=L, B=B, centre=centre, scale=scale, rays_o=o,
                        rays_d=d, t=t, depth=depth, rgb=rgb, mask=mask)
    raise RuntimeError("no smooth problem found")


def loss_of(pb, theta):
    loss, _, _ = oracle.object_loss_and_grad(theta, pb["H"], pb["L"], pb["B"], pb["centre"],
                                             pb["scale"], pb["rays_o"], pb["rays_d"], pb["t"],
                                             pb["depth"], pb["rgb"], pb["mask"], want_grad=False)
    return loss


def grad_of(pb, theta, upstream=1.0):
    return oracle.object_loss_and_grad(theta, pb["H"], pb["L"], pb["B"], pb["centre"],
                                       pb["scale"], pb["rays_o"], pb["rays_d"], pb["t"],
                                       pb["depth"], pb["rgb"], pb["mask"], upstream=upstream)


# ----------------------------------------------------------------------------- constants

def test_paper_constants():
    g = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    assert oracle.LAMBDA_COLOUR == g["lambda_colour"]["value"]
    assert oracle.LAMBDA_OCC == g["lambda_occupancy"]["value"]
    assert scenes.WORKLOADS["tiny_k4"]["near"] == ("normal", g["d_sigma_m"]["value"])
    assert scenes.WORKLOADS["tiny_k4"]["rays"] == ("fixed", g["object_rays_per_step"]["value"])
    assert scenes.WORKLOADS["tiny_k4"]["S"] == g["points_per_ray"]["value"]
    assert scenes.WORKLOADS["tiny_k4"]["hidden"] == g["object_hidden"]["value"]
    bg = scenes.WORKLOADS["room50_background"]["background"]
    assert bg == dict(hidden=g["background_hidden"]["value"],
                      rays=g["background_rays_per_step"]["value"])


# ----------------------------------------------------------------------------- initialisation

def test_splitmix64_published_vector():
    # First five outputs of SplitMix64 seeded with 1234567, as printed by the reference C
    # implementation that accompanies Steele, Lea and Flood (2014) / Vigna's splitmix64.c.
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    got = oracle.splitmix64(1234567, np.arange(5))
    assert [int(x) for x in got] == want


def test_xavier_init_bounds_and_moments():
    H, L, E = 64, 4, 32
    theta = oracle.xavier_init(12345, H, L, E).astype(np.float64)
    assert theta.dtype == np.float64 and theta.shape == (oracle.n_params(H, L, E),)
    for (W, b), (o, i) in zip(oracle.unpack(theta, H, L, E), oracle.layer_shapes(H, L, E)):
        a = math.sqrt(6.0 / (i + o))
        assert np.all(b == 0.0)
        assert np.max(np.abs(W)) <= a
        n = W.size
        # U(-a, a): mean 0, variance a^2 / 3; 5-sigma bands
        assert abs(W.mean()) < 5 * a / math.sqrt(3 * n)
        var = W.var()
        assert abs(var - a * a / 3) < 5 * (a * a) * math.sqrt(4 / 45 / n)
    # different seeds give different models, the same seed the same model
    assert not np.array_equal(oracle.xavier_init(1, H, L, E), oracle.xavier_init(2, H, L, E))
    assert np.array_equal(oracle.xavier_init(7, H, L, E), oracle.xavier_init(7, H, L, E))


def test_param_counts():
    # E = 32 inputs, four hidden layers, four outputs
    assert oracle.n_params(32, 4, 32) == 4356
    assert oracle.n_params(64, 4, 32) == 14852
    assert oracle.n_params(128, 4, 32) == 54276
    assert oracle.n_params(8, 0, 32) == 4 * 32 + 4       # linear model


# ----------------------------------------------------------------------------- encoding

def test_encoding_at_origin():
    B = np.random.default_rng(0).normal(0, 5, size=(3, 16))
    g = oracle.encode(np.zeros((1, 3)), B)
    np.testing.assert_array_equal(g[0, :16], 0.0)
    np.testing.assert_array_equal(g[0, 16:], 1.0)


def test_encoding_unit_columns_gives_coordinate_sines():
    B = np.zeros((3, 16))
    B[0, 0] = B[1, 1] = B[2, 2] = 1.0
    x = np.array([[0.3, -0.7, 1.1]])
    g = oracle.encode(x, B)
    np.testing.assert_allclose(g[0, :3], np.sin(x[0]), rtol=0, atol=1e-15)
    np.testing.assert_allclose(g[0, 16:19], np.cos(x[0]), rtol=0, atol=1e-15)
    np.testing.assert_array_equal(g[0, 3:16], 0.0)
    np.testing.assert_array_equal(g[0, 19:], 1.0)


def test_normalisation_maps_bound_to_unit_box():
    sc = scenes.make_scene("k50_uneven")
    for ob in sc.objects[:10]:
        corners = np.array([[x, y, z] for x in (ob.bound_lo[0], ob.bound_hi[0])
                            for y in (ob.bound_lo[1], ob.bound_hi[1])
                            for z in (ob.bound_lo[2], ob.bound_hi[2])])
        x = oracle.normalise(corners, np.zeros_like(corners), np.zeros((8, 1)), ob.norm_centre,
                             ob.norm_scale)
        assert np.max(np.abs(x)) == pytest.approx(1.0, abs=1e-12)


# ----------------------------------------------------------------------------- MLP

def test_mlp_forward_matches_torch_linear():
    rng = np.random.default_rng(3)
    H, L, E = 16, 3, 32
    theta = rng.normal(size=oracle.n_params(H, L, E))
    gamma = rng.normal(size=(50, E))
    z, pre = oracle.mlp_forward(theta, gamma, H, L)
    net = []
    for (W, b) in oracle.unpack(theta, H, L, E):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W.copy()))
            lin.bias.copy_(torch.from_numpy(b.copy()))
        net += [lin, torch.nn.ReLU()]
    ref = torch.nn.Sequential(*net[:-1])(torch.from_numpy(gamma)).detach().numpy()
    np.testing.assert_allclose(z, ref, rtol=1e-13, atol=1e-13)
    assert len(pre) == L


# ----------------------------------------------------------------------------- rendering

def _object_with_constant_heads(occ, colour, H=8, L=2, F=4, seed=0):
    rng = np.random.default_rng(seed)
    theta = rng.normal(size=oracle.n_params(H, L, 2 * F))
    W, b = oracle.unpack(theta, H, L, 2 * F)[-1]
    W[:] = 0.0
    b[:3] = np.log(np.asarray(colour) / (1 - np.asarray(colour)))
    b[3] = math.log(occ / (1 - occ))
    return theta, H, L, rng.normal(size=(3, F))


@pytest.mark.parametrize("occ,S", [(0.3, 10), (0.05, 20), (0.9, 7), (0.5, 1)])
def test_render_constant_occupancy_closed_form(occ, S):
    colour = np.array([0.2, 0.5, 0.9])
    theta, H, L, B = _object_with_constant_heads(occ, colour)
    R = 5
    rng = np.random.default_rng(1)
    a = rng.uniform(1.0, 2.0, size=R)
    delta = rng.uniform(0.01, 0.2, size=R)
    t = a[:, None] + delta[:, None] * np.arange(S)[None, :]
    o = np.tile([0.0, 0.0, -3.0], (R, 1))
    d = np.tile([0.0, 0.0, 1.0], (R, 1))
    fw = oracle.object_forward(theta, H, L, B, np.zeros(3), 1.0, o, d, t)
    q = 1.0 - occ
    O = np.full(R, 1.0 - q ** S)
    D = a * O + delta * occ * q * (1 - S * q ** (S - 1) + (S - 1) * q ** S) / (1 - q) ** 2
    np.testing.assert_allclose(fw["O"], O, rtol=1e-13)
    np.testing.assert_allclose(fw["D"], D, rtol=1e-13)
    np.testing.assert_allclose(fw["C"], O[:, None] * colour[None, :], rtol=1e-13)
    # termination probabilities are geometric
    np.testing.assert_allclose(fw["T"], occ * q ** np.arange(S)[None, :].repeat(R, 0),
                               rtol=1e-13)


def test_render_brute_force_product():
    rng = np.random.default_rng(5)
    R, S = 7, 13
    o = rng.uniform(size=(R, S))
    c = rng.uniform(size=(R, S, 3))
    t = np.sort(rng.uniform(1, 5, size=(R, S)), axis=1)
    O, D, C, T, P = oracle.render(o, c, t)
    for r in range(R):
        Tb = [o[r, i] * np.prod([1 - o[r, j] for j in range(i)]) for i in range(S)]
        assert O[r] == pytest.approx(sum(Tb), rel=1e-14)
        assert D[r] == pytest.approx(sum(Tb[i] * t[r, i] for i in range(S)), rel=1e-14)
        for k in range(3):
            assert C[r, k] == pytest.approx(sum(Tb[i] * c[r, i, k] for i in range(S)), rel=1e-14)
        assert P[r, S] == pytest.approx(np.prod(1 - o[r]), rel=1e-14)


def test_render_special_cases():
    rng = np.random.default_rng(6)
    S = 6
    c = rng.uniform(size=(1, S, 3))
    t = np.sort(rng.uniform(1, 5, size=(1, S)), axis=1)
    # first sample fully occupied: everything comes from it
    o = rng.uniform(size=(1, S))
    o[0, 0] = 1.0
    O, D, C, _, _ = oracle.render(o, c, t)
    assert O[0] == 1.0 and D[0] == t[0, 0]
    np.testing.assert_array_equal(C[0], c[0, 0])
    # empty space renders nothing
    O, D, C, _, _ = oracle.render(np.zeros((1, S)), c, t)
    assert O[0] == 0.0 and D[0] == 0.0 and np.all(C == 0.0)
    # one sample: O = o_1
    O, D, C, _, _ = oracle.render(np.array([[0.37]]), c[:, :1], t[:, :1])
    assert O[0] == 0.37 and D[0] == pytest.approx(0.37 * t[0, 0])


def test_render_vjp_closed_form():
    rng = np.random.default_rng(8)
    R, S = 4, 9
    o = rng.uniform(size=(R, S))
    c = rng.uniform(size=(R, S, 3))
    t = np.sort(rng.uniform(1, 5, size=(R, S)), axis=1)
    one, zero = np.ones(R), np.zeros(R)
    do, dc = oracle.render_vjp(o, c, t, one, zero, np.zeros((R, 3)), zero)
    # dO/do_i = prod_{j != i} (1 - o_j)
    want = np.array([[np.prod(np.delete(1 - o[r], i)) for i in range(S)] for r in range(R)])
    np.testing.assert_allclose(do, want, rtol=1e-12)
    np.testing.assert_array_equal(dc, 0.0)
    # d P_{S+1} / d o_i = -prod_{j != i} (1 - o_j)
    do, _ = oracle.render_vjp(o, c, t, zero, zero, np.zeros((R, 3)), one)
    np.testing.assert_allclose(do, -want, rtol=1e-12)
    # depth and colour cotangents: compare with central differences of render itself
    gD = rng.normal(size=R)
    gC = rng.normal(size=(R, 3))
    do, dc = oracle.render_vjp(o, c, t, zero, gD, gC, zero)
    h = 1e-6
    for i in range(S):
        op, om = o.copy(), o.copy()
        op[:, i] += h
        om[:, i] -= h
        _, Dp, Cp, _, _ = oracle.render(op, c, t)
        _, Dm, Cm, _, _ = oracle.render(om, c, t)
        fd = gD * (Dp - Dm) / (2 * h) + np.sum(gC * (Cp - Cm), axis=1) / (2 * h)
        np.testing.assert_allclose(do[:, i], fd, rtol=1e-7, atol=1e-9)
    _, _, _, T, _ = oracle.render(o, c, t)
    np.testing.assert_allclose(dc, T[:, :, None] * gC[:, None, :], rtol=1e-14)


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 32), st.integers(0, 2 ** 31 - 1))
def test_render_invariants(S, seed):
    rng = np.random.default_rng(seed)
    R = 6
    o = rng.uniform(size=(R, S)) ** rng.uniform(0.2, 4)
    c = rng.uniform(size=(R, S, 3))
    t = np.sort(rng.uniform(0.1, 8, size=(R, S)), axis=1)
    O, D, C, T, P = oracle.render(o, c, t)
    assert np.all(T >= 0)
    np.testing.assert_allclose(T.sum(1), 1.0 - P[:, S], rtol=1e-12, atol=1e-15)
    assert np.all(O <= 1.0 + 1e-15)
    assert np.all(O * t[:, 0] <= D * (1 + 1e-12) + 1e-300)
    assert np.all(D <= O * t[:, -1] * (1 + 1e-12) + 1e-300)
    assert np.all(C >= 0) and np.all(C <= O[:, None] * (1 + 1e-12) + 1e-300)


# ----------------------------------------------------------------------------- loss + gradient

def test_loss_hand_example():
    """One ray, S = 2, constant occupancy 1/2 and colour 1/4, worked by hand from Eqs. 3-7.

    T = (1/2, 1/4); O = 3/4; D = t1/2 + t2/4; C = 3/16 per channel; 1 - O = 1/4.
    """
    theta, H, L, B = _object_with_constant_heads(0.5, [0.25, 0.25, 0.25])
    t = np.array([[2.0, 3.0]])
    o = np.array([[0.0, 0.0, -3.0]])
    d = np.array([[0.0, 0.0, 1.0]])
    args = (theta, H, L, B, np.zeros(3), 1.0, o, d, t)
    # inside the mask: depth 1.5, colour (1, 0, 0.5)
    loss, _, _ = oracle.object_loss_and_grad(*args, np.array([1.5]), np.array([[1, 0, 0.5]]),
                                             np.array([1.0]), want_grad=False)
    D = 2.0 / 2 + 3.0 / 4
    colour = abs(3 / 16 - 1) + abs(3 / 16 - 0) + abs(3 / 16 - 0.5)
    assert loss == pytest.approx(abs(D - 1.5) + 5 * colour + 10 * 0.25, rel=1e-13)
    # outside the mask: only the occupancy term, |O - 0| = 3/4
    loss, _, _ = oracle.object_loss_and_grad(*args, np.array([1.5]), np.array([[1, 0, 0.5]]),
                                             np.array([0.0]), want_grad=False)
    assert loss == pytest.approx(10 * 0.75, rel=1e-13)


@pytest.mark.parametrize("seed,H,L,F,S", [(0, 4, 2, 3, 4), (1, 5, 1, 2, 3), (2, 3, 0, 2, 5),
                                         (3, 4, 3, 3, 1)])
def test_gradient_central_differences(seed, H, L, F, S):
    pb = tiny_problem(seed, S=S, H=H, L=L, F=F)
    loss, g, _ = grad_of(pb, pb["theta"])
    h = 1e-6
    fd = np.empty_like(g)
    for p in range(g.size):
        tp, tm = pb["theta"].copy(), pb["theta"].copy()
        tp[p] += h
        tm[p] -= h
        fd[p] = (loss_of(pb, tp) - loss_of(pb, tm)) / (2 * h)
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(fd)
    # the upstream weight scales the gradient linearly
    _, g3, _ = grad_of(pb, pb["theta"], upstream=-3.0)
    np.testing.assert_allclose(g3, -3.0 * g, rtol=1e-13, atol=1e-15)


def _torch_loss(pb, theta_t):
    """The same objective written in torch ops; torch's autograd supplies the gradient."""
    H, L = pb["H"], pb["L"]
    f64 = torch.float64
    o = torch.tensor(pb["rays_o"], dtype=f64)[:, None, :]
    d = torch.tensor(pb["rays_d"], dtype=f64)[:, None, :]
    t = torch.tensor(pb["t"], dtype=f64)
    x = (o + t[:, :, None] * d - torch.tensor(pb["centre"], dtype=f64)) / pb["scale"]
    phi = x @ torch.tensor(pb["B"], dtype=f64)
    h = torch.cat([torch.sin(phi), torch.cos(phi)], -1)
    E = h.shape[-1]
    widths = [E] + [H] * L + [4]
    off = 0
    for li in range(len(widths) - 1):
        fo, fi = widths[li + 1], widths[li]
        W = theta_t[off:off + fo * fi].reshape(fo, fi)
        off += fo * fi
        b = theta_t[off:off + fo]
        off += fo
        h = h @ W.T + b
        if li < len(widths) - 2:
            h = torch.relu(h)
    c = torch.sigmoid(h[..., :3])
    occ = torch.sigmoid(h[..., 3])
    keep = torch.cumprod(1 - occ, dim=1)
    excl = torch.cat([torch.ones_like(keep[:, :1]), keep[:, :-1]], 1)
    T = occ * excl
    O, D, C = T.sum(1), (T * t).sum(1), (T[:, :, None] * c).sum(1)
    M = torch.tensor(pb["mask"], dtype=f64)
    rho = torch.where(M == 1, -keep[:, -1], O - M)
    return (M * (D - torch.tensor(pb["depth"], dtype=f64)).abs()).sum() \
        + 5 * (M[:, None] * (C - torch.tensor(pb["rgb"], dtype=f64)).abs()).sum() \
        + 10 * rho.abs().sum()


@pytest.mark.parametrize("seed", range(4))
def test_gradient_matches_torch_autograd(seed):
    pb = tiny_problem(100 + seed, R=6, S=7, H=8, L=4, F=4)
    loss, g, _ = grad_of(pb, pb["theta"])
    th = torch.tensor(pb["theta"], dtype=torch.float64, requires_grad=True)
    lt = _torch_loss(pb, th)
    lt.backward()
    assert loss == pytest.approx(lt.item(), rel=1e-13)
    np.testing.assert_allclose(g, th.grad.numpy(), rtol=1e-10, atol=1e-12)


# ----------------------------------------------------------------------------- Adam

def test_adam_first_step_closed_form():
    rng = np.random.default_rng(9)
    theta = rng.normal(size=100)
    g = rng.normal(size=100) * 10.0 ** rng.uniform(-6, 2, size=100)
    th1, m, v = oracle.adam_update(theta, np.zeros(100), np.zeros(100), g, 1)
    np.testing.assert_allclose(th1, theta - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    assert np.all(np.abs(th1 - theta) < 1e-3)


def test_adam_second_step_values():
    g1, g2 = np.array([0.5, -2.0]), np.array([1.5, 1.0])
    th = np.array([1.0, -1.0])
    th1, m, v = oracle.adam_update(th, np.zeros(2), np.zeros(2), g1, 1)
    th2, m, v = oracle.adam_update(th1, m, v, g2, 2)
    np.testing.assert_allclose(m, 0.09 * g1 + 0.1 * g2, rtol=1e-15)
    np.testing.assert_allclose(v, 0.000999 * g1 ** 2 + 0.001 * g2 ** 2, rtol=1e-14)
    m_hat = m / 0.19
    v_hat = v / 0.001999
    np.testing.assert_allclose(th2, th1 - 1e-3 * m_hat / (np.sqrt(v_hat) + 1e-8), rtol=1e-14)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(10)
    theta = rng.normal(size=64)
    p = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(64)
    v = np.zeros(64)
    for k in range(1, 6):
        g = rng.normal(size=64)
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        theta, m, v = oracle.adam_update(theta, m, v, g, k)
    np.testing.assert_allclose(theta, p.detach().numpy(), rtol=1e-13, atol=1e-15)


# ----------------------------------------------------------------------------- whole step

def _states(scene, ids=None):
    ids = range(scene.n_objects) if ids is None else ids
    out = {}
    for k in ids:
        ob = scene.objects[k]
        th = oracle.xavier_init(ob.seed, ob.hidden, 4, 32)
        out[k] = oracle.ObjectState(th, ob.hidden, 4, ob.norm_centre, ob.norm_scale)
    return out


def _sub(batch, js):
    """Sub-batch of the listed batch positions, in that order."""
    offs = batch["ray_offsets"]
    rows = np.concatenate([np.arange(offs[j], offs[j + 1]) for j in js]).astype(np.int64)
    counts = [offs[j + 1] - offs[j] for j in js]
    out = {k: batch[k][rows] for k in ("rays_o", "rays_d", "t", "depth", "rgb", "mask")}
    out["object_ids"] = batch["object_ids"][list(js)]
    out["ray_offsets"] = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    out["S"] = batch["S"]
    return out


def test_step_permutation_split_and_zero_rays():
    sc = scenes.make_scene("tiny_k4")
    batch = scenes.make_batch(sc, 0)
    base = _states(sc)
    s0 = {k: v.copy() for k, v in base.items()}
    l0, g0, r0 = oracle.step(s0, batch, sc.B)
    # permuting objects permutes every result
    perm = [2, 0, 3, 1]
    s1 = {k: v.copy() for k, v in base.items()}
    l1, g1, _ = oracle.step(s1, _sub(batch, perm), sc.B)
    np.testing.assert_array_equal(l1, l0[perm])
    for k in range(4):
        np.testing.assert_array_equal(g1[k], g0[k])
        np.testing.assert_array_equal(s1[k].theta, s0[k].theta)
    # splitting the batch changes nothing
    s2 = {k: v.copy() for k, v in base.items()}
    la, _, _ = oracle.step(s2, _sub(batch, [0, 1]), sc.B)
    lb, _, _ = oracle.step(s2, _sub(batch, [2, 3]), sc.B)
    np.testing.assert_array_equal(np.concatenate([la, lb]), l0)
    for k in range(4):
        np.testing.assert_array_equal(s2[k].theta, s0[k].theta)
        assert s2[k].t == 1
    # an object with zero rays is untouched (parameters, moments and step count)
    s3 = {k: v.copy() for k, v in base.items()}
    zb = scenes.make_batch(sc, 0, n_rays={1: 0})
    l3, _, _ = oracle.step(s3, zb, sc.B)
    assert l3[1] == 0.0 and s3[1].t == 0
    np.testing.assert_array_equal(s3[1].theta, base[1].theta)
    np.testing.assert_array_equal(s3[1].m, 0.0)
    np.testing.assert_array_equal(s3[1].v, 0.0)
    for k in (0, 2, 3):
        np.testing.assert_array_equal(s3[k].theta, s0[k].theta)


def test_step_renders_and_losses_are_consistent():
    sc = scenes.make_scene("tiny_k4")
    batch = scenes.make_batch(sc, 0)
    st_ = _states(sc)
    losses, grads, rend = oracle.step(st_, batch, sc.B, apply_adam=False)
    offs = batch["ray_offsets"]
    for j in range(4):
        sl = slice(offs[j], offs[j + 1])
        M = batch["mask"][sl].astype(np.float64)
        want = np.sum(M * np.abs(rend["D"][sl] - batch["depth"][sl]))
        want += 5 * np.sum(M[:, None] * np.abs(rend["C"][sl] - batch["rgb"][sl]))
        want += 10 * np.sum(np.abs(rend["O"][sl] - M))
        # |O - M| and |rho| agree up to the rounding of O itself
        assert losses[j] == pytest.approx(want, rel=1e-9)
    assert all(st_[k].t == 0 for k in st_)


def test_query_matches_forward_samples():
    sc = scenes.make_scene("tiny_k4")
    batch = scenes.make_batch(sc, 0)
    ob = sc.objects[0]
    th = oracle.xavier_init(ob.seed, 32, 4, 32)
    r1 = batch["ray_offsets"][1]
    fw = oracle.object_forward(th, 32, 4, sc.B, ob.norm_centre, ob.norm_scale,
                               batch["rays_o"][:r1], batch["rays_d"][:r1], batch["t"][:r1])
    pts = (batch["rays_o"][:r1, None, :].astype(np.float64)
           + batch["t"][:r1, :, None] * batch["rays_d"][:r1, None, :].astype(np.float64))
    occ, rgb = oracle.query(th, 32, 4, sc.B, ob.norm_centre, ob.norm_scale, pts.reshape(-1, 3))
    np.testing.assert_allclose(occ, fw["o"].ravel(), rtol=1e-12)
    np.testing.assert_allclose(rgb, fw["c"].reshape(-1, 3), rtol=1e-12)


# ----------------------------------------------------------------------------- sampling

def test_splitmix64_array_matches_scalar_definition():
    idx = np.array([0, 1, 2, 1000, 2 ** 40 + 3], dtype=np.uint64)
    for seed in (0, 1234567, 2 ** 64 - 1):
        np.testing.assert_array_equal(oracle.splitmix64_array(seed, idx),
                                      oracle.splitmix64(seed, idx.astype(np.int64)))


def test_depth_guided_samples_properties():
    """Eq. 1: each stratified sample lies in its own stratum of [t_n, t_s]; Eq. 2: the surface
    samples have mean t_s and spread sigma; t_s falls back to t_f for invalid depth."""
    rng = np.random.default_rng(0)
    R, S, Nc, sigma = 4000, 20, 10, 0.03
    tn = rng.uniform(0.5, 1.0, R)
    tf = tn + rng.uniform(1.0, 3.0, R)
    depth = np.where(rng.uniform(size=R) < 0.8, rng.uniform(tn + 0.2, tf), 0.0)
    t = oracle.depth_guided_samples(tn, tf, depth, S, Nc, sigma, seed=42)
    assert t.shape == (R, S) and np.all(np.diff(t, axis=1) >= 0)
    # rebuild the unsorted samples to check each stratum
    ts = np.where(depth > 0, depth, tf)
    idx = (np.arange(R)[:, None] * S + np.arange(S)[None, :]).astype(np.uint64) * np.uint64(2)
    u = (oracle.splitmix64_array(42, idx) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    for i in range(Nc):
        lo = tn + i / Nc * (ts - tn)
        hi = tn + (i + 1) / Nc * (ts - tn)
        x = tn + (i + u[:, i]) / Nc * (ts - tn)
        assert np.all(x >= lo - 1e-12) and np.all(x <= hi + 1e-12)
        # each stratified value appears among the sorted samples of its ray
        assert np.all(np.min(np.abs(t - x[:, None]), axis=1) < 1e-12)
    # surface samples: the S - Nc values not matched to strata, z-scored
    strat = np.stack([tn + (i + u[:, i]) / Nc * (ts - tn) for i in range(Nc)], 1)
    z = []
    for r in range(R):
        rest = list(t[r])
        for x in strat[r]:
            rest.pop(int(np.argmin(np.abs(np.array(rest) - x))))
        z.extend((np.array(rest) - ts[r]) / sigma)
    z = np.array(z)
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1.0) < 0.02


# ------------------------------------------------------------------------ scene rendering

def test_ray_box_against_brute_force():
    """Slab entry/exit against dense point sampling of each ray (including directions with a
    zero component, origins inside the box and rays that miss)."""
    rng = np.random.default_rng(11)
    ts = np.linspace(-12.0, 12.0, 240001)
    step = ts[1] - ts[0]
    for trial in range(120):
        lo = rng.uniform(-1.0, 0.0, 3)
        hi = lo + rng.uniform(0.1, 1.5, 3)
        o = rng.uniform(-3.0, 3.0, 3) if trial % 5 else rng.uniform(lo, hi)
        d = rng.standard_normal(3)
        if trial % 7 == 0:
            d[trial % 3] = 0.0
        d /= np.linalg.norm(d)
        t0, t1 = oracle.ray_box(o[None], d[None], lo, hi)
        pts = o[None, :] + ts[:, None] * d[None, :]
        inside = np.all((pts >= lo) & (pts <= hi), axis=1)
        if inside.any():
            assert abs(t0[0] - ts[inside][0]) <= step and abs(t1[0] - ts[inside][-1]) <= step
        else:
            assert t1[0] < t0[0] + step


def _constant_model(H, colour, occ, seed=3):
    """Parameters whose outputs are constant: zero output weights, logits in the output bias."""
    th = oracle.xavier_init(seed, H, 4, 32).astype(np.float64)
    logit = lambda p: np.log(p / (1.0 - p))
    th[-(4 * H + 4):-4] = 0.0
    th[-4:] = [logit(colour[0]), logit(colour[1]), logit(colour[2]), logit(occ)]
    return th


def _constant_render(o, t):
    """Closed form of Eq. 3 for constant occupancy o at depths t: T_i = o (1 - o)^(i-1)."""
    q = 1.0 - o
    w = o * q ** np.arange(len(t))
    return 1.0 - q ** len(t), float(np.sum(w * t))


def test_render_scene_ranks_constant_occupancy_objects():
    """Two boxes on one ray with constant outputs: the nearer one wins while its rendered
    occupancy reaches the threshold, the farther one otherwise; a ray that meets neither box
    gets no object."""
    H, S = 32, 8
    B = np.random.default_rng(1).normal(0.0, 5.0, (3, 16))
    cA, cB = np.array([0.3, 0.6, 0.1]), np.array([0.9, 0.2, 0.5])
    o_rays = np.array([[0.1, -0.1, -5.0], [0.0, 5.0, 0.0]])
    d_rays = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    for oA, oB, winner in ((0.3, 0.4, 0), (0.02, 0.4, 1), (0.02, 0.05, -1)):
        sA = oracle.ObjectState(_constant_model(H, cA, oA), H, 4, np.zeros(3), 0.5)
        sB = oracle.ObjectState(_constant_model(H, cB, oB), H, 4, np.array([0.0, 0.0, 2.0]), 0.5)
        depth, rgb, occ, k = oracle.render_scene([sA, sB], B, o_rays, d_rays, S)
        assert k[1] == -1 and depth[1] == 0.0 and np.all(rgb[1] == 0.0)
        assert k[0] == winner
        if winner < 0:
            continue
        t0, t1 = (4.5, 5.5) if winner == 0 else (6.5, 7.5)
        t = (t0 + (np.arange(S) + 0.5) / S * (t1 - t0)).astype(np.float32).astype(np.float64)
        O, D = _constant_render(oA if winner == 0 else oB, t)
        col = cA if winner == 0 else cB
        assert abs(occ[0] - O) <= 1e-12 and abs(depth[0] - D) <= 1e-12
        np.testing.assert_allclose(rgb[0], O * col, rtol=1e-12)
        assert O >= 0.5


# ------------------------------------------------------------------------ integrated encoding

def test_integrated_encoding_is_the_gaussian_expectation():
    """Monte Carlo: the mean of [sin(x B), cos(x B)] over x ~ N(mu, var I) matches the closed
    form within five standard errors; var = 0 gives the point encoding bit for bit."""
    rng = np.random.default_rng(21)
    B = rng.normal(0.0, 5.0, (3, 16)) * 0.2
    for mu, var in ((np.array([0.1, -0.3, 0.5]), 0.05), (np.array([-0.7, 0.2, 0.0]), 0.3)):
        n = 400_000
        xs = mu[None, :] + np.sqrt(var) * rng.standard_normal((n, 3))
        phi = xs @ B
        mc = np.concatenate([np.sin(phi), np.cos(phi)], axis=1)
        mean, se = mc.mean(0), mc.std(0) / np.sqrt(n)
        got = oracle.encode(mu[None, :], B, np.array([var]))[0]
        assert np.all(np.abs(got - mean) <= 5 * se + 1e-12), np.max(np.abs(got - mean) / se)
    x = rng.uniform(-1, 1, (50, 3))
    assert np.array_equal(oracle.encode(x, B, np.zeros(50)), oracle.encode(x, B))
