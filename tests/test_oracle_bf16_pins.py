"""Pins of the oracle's BF16 modes against torch (CPU), independently of the oracle's own code.

The BF16 form (not in the paper) rounds every operand of every MLP product to BF16, round to
nearest even, and accumulates in FP32; the oracle's diagnostic mode does the same rounding with
FP64 accumulation. Three things are pinned here:

* ``oracle.bf16_round`` against torch's float32 -> bfloat16 cast over ties, near-ties, signed
  zeros, subnormals, the overflow boundary, infinities, NaN payloads and random bit patterns;
* the ``rnd`` path of ``oracle.object_loss_and_grad`` against a float64 torch objective written
  here from the same readings (Eqs. 3-7 with the build's encoding and MLP), whose linear layers
  round their operands with torch's bfloat16 cast in forward and backward (a custom autograd
  function: every product of the MLP takes rounded operands, the output layer's seed dz
  included; bias gradients sum the rounded deltas except at the output layer);
* the ``decide`` path: the ReLU decisions and L1 signs of the BF16 forward, the arithmetic in
  FP64, against torch autograd of the objective with those pieces fixed (ReLU replaced by a
  multiplication with the decided mask, |r| by s r with the decided sign).
"""
import numpy as np
import pytest
import torch

import oracle

F64 = torch.float64


def tb(x):
    """torch's own rounding to BF16 (float64 -> float32 -> bfloat16), back to float64."""
    return x.to(torch.float32).to(torch.bfloat16).to(F64)


# ----------------------------------------------------------------------------- rounding

def _special_patterns():
    p = []
    for hi in (0x3F80, 0x3F81, 0x4049, 0x404A, 0x0001, 0x0080, 0x7F7E, 0x7F7F):
        for lo in (0x0000, 0x0001, 0x7FFF, 0x8000, 0x8001, 0xFFFF):
            p.append((hi << 16) | lo)
    p += [0x00000000, 0x00000001, 0x00007FFF, 0x00008000, 0x00018000, 0x007FFFFF,  # +0, subnormals
          0x7F7FFFFF, 0x7F7F8000, 0x7F7F7FFF,                                    # overflow edge
          0x7F800000,                                                            # +inf
          0x7F800001, 0x7F807FFF, 0x7F808000, 0x7FBFFFFF, 0x7FC00000, 0x7FFFFFFF]  # NaN payloads
    p += [x | 0x80000000 for x in p]                                             # and negatives
    return np.array(p, dtype=np.uint32)


def test_bf16_round_matches_torch_cast():
    rng = np.random.default_rng(11)
    bits = np.concatenate([_special_patterns(),
                           rng.integers(0, 1 << 32, size=200_000, dtype=np.uint64).astype(np.uint32)])
    x = bits.view(np.float32)
    got = oracle.bf16_round(x)
    want = tb(torch.from_numpy(x.copy())).numpy()
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan].view(np.uint64), want[~nan].view(np.uint64))  # signed zeros too
    # FP64 inputs go through FP32 first, as in the kernels (FP32 values rounded to BF16)
    y = rng.standard_normal(50_000) * np.exp(rng.uniform(-30, 30, size=50_000))
    assert np.array_equal(oracle.bf16_round(y), tb(torch.from_numpy(y)).numpy())
    # shape is kept, scalars included
    assert oracle.bf16_round(np.float64(1.0 + 2.0 ** -9)).shape == ()
    assert oracle.bf16_round(np.ones((2, 3))).shape == (2, 3)


# ----------------------------------------------------------------------------- objective

class _BLinear(torch.autograd.Function):
    """y = bf16(x) bf16(W)^T + b; backward rounds dy, W and x where they enter products."""

    @staticmethod
    def forward(ctx, x, W, b, head):
        ctx.save_for_backward(x, W)
        ctx.head = head
        return tb(x) @ tb(W).T + b

    @staticmethod
    def backward(ctx, dy):
        x, W = ctx.saved_tensors
        d = tb(dy)
        db = (dy if ctx.head else d).sum(0)
        return d @ tb(W), d.T @ tb(x), db, None


def _problem(seed, R=24, S=6, H=16, L=3, F=4):
    rng = np.random.default_rng(seed)
    E = 2 * F
    theta = np.concatenate([np.concatenate([rng.uniform(-1, 1, size=o * i) * np.sqrt(6.0 / (o + i)),
                                            rng.normal(0, 0.1, size=o)])
                            for o, i in oracle.layer_shapes(H, L, E)])
    o = rng.normal(0.0, 1.0, size=(R, 3)) + np.array([0.0, 0.0, -3.0])
    d = rng.normal(0.0, 0.2, size=(R, 3)) + np.array([0.0, 0.0, 1.0])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return dict(theta=theta, H=H, L=L, B=rng.normal(0.0, 2.0, size=(3, F)),
                centre=rng.normal(0.0, 0.3, size=3), scale=rng.uniform(0.5, 1.5), rays_o=o,
                rays_d=d, t=np.sort(rng.uniform(2.0, 4.0, size=(R, S)), axis=1),
                depth=rng.uniform(2.0, 4.0, size=R), rgb=rng.uniform(0.0, 1.0, size=(R, 3)),
                mask=(rng.uniform(size=R) < 0.6).astype(np.float64))


def _torch_loss(pb, mode, decisions=None):
    """The loss of Eqs. 3-7 in torch float64 with parameters as leaves.

    mode "bf16": BF16 operands in every MLP product (custom autograd above);
    mode "fixed": FP64, ReLU and L1 pieces fixed by ``decisions`` = (relu masks, signs).
    Returns (loss, leaves, decisions of this forward)."""
    H, L = pb["H"], pb["L"]
    E = 2 * pb["B"].shape[1]
    leaves, off = [], 0
    th = torch.tensor(pb["theta"], dtype=F64)
    for o, i in oracle.layer_shapes(H, L, E):
        W = th[off:off + o * i].reshape(o, i).clone().requires_grad_(True)
        off += o * i
        b = th[off:off + o].clone().requires_grad_(True)
        off += o
        leaves += [W, b]
    ro = torch.tensor(pb["rays_o"], dtype=F64)
    rd = torch.tensor(pb["rays_d"], dtype=F64)
    t = torch.tensor(pb["t"], dtype=F64)
    R, S = t.shape
    x = (ro[:, None, :] + t[:, :, None] * rd[:, None, :] - torch.tensor(pb["centre"], dtype=F64)) \
        / pb["scale"]
    phi = x.reshape(R * S, 3) @ torch.tensor(pb["B"], dtype=F64)
    h = torch.cat([torch.sin(phi), torch.cos(phi)], dim=1)
    masks = []
    n_lin = len(leaves) // 2
    for li in range(n_lin):
        W, b = leaves[2 * li], leaves[2 * li + 1]
        head = li == n_lin - 1
        a = _BLinear.apply(h, W, b, head) if mode == "bf16" else h @ W.T + b
        if head:
            z = a
            break
        masks.append((a > 0).detach())
        h = torch.relu(a) if mode == "bf16" else a * decisions[0][li].to(F64)
    o = torch.sigmoid(z[:, 3]).reshape(R, S)
    c = torch.sigmoid(z[:, :3]).reshape(R, S, 3)
    P = torch.cumprod(torch.cat([torch.ones(R, 1, dtype=F64), 1.0 - o], dim=1), dim=1)
    T = o * P[:, :S]
    O_, D_, C_ = T.sum(1), (T * t).sum(1), (T[:, :, None] * c).sum(1)
    M = torch.tensor(pb["mask"], dtype=F64)
    rD = D_ - torch.tensor(pb["depth"], dtype=F64)
    rC = C_ - torch.tensor(pb["rgb"], dtype=F64)
    rho = torch.where(M == 1.0, -P[:, S], O_ - M)
    signs = (torch.sign(rD).detach(), torch.sign(rC).detach(), torch.sign(rho).detach())
    if mode == "bf16":
        loss = (M * rD.abs()).sum() + 5.0 * (M[:, None] * rC.abs()).sum() + 10.0 * rho.abs().sum()
    else:
        sD, sC, sR = decisions[1]
        loss = (M * sD * rD).sum() + 5.0 * (M[:, None] * sC * rC).sum() + 10.0 * (sR * rho).sum()
    return loss, leaves, (masks, signs)


def _oracle_grad(pb, **kw):
    return oracle.object_loss_and_grad(pb["theta"], pb["H"], pb["L"], pb["B"], pb["centre"],
                                       pb["scale"], pb["rays_o"], pb["rays_d"], pb["t"],
                                       pb["depth"], pb["rgb"], pb["mask"], **kw)


def _flat(leaves):
    return np.concatenate([p.grad.numpy().ravel() for p in leaves])


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bf16_mode_gradient_matches_torch_objective(seed):
    pb = _problem(seed)
    loss_t, leaves, _ = _torch_loss(pb, "bf16")
    loss_t.backward()
    g_t = _flat(leaves)
    loss_o, g_o, _ = _oracle_grad(pb, rnd=oracle.bf16_round)
    assert abs(loss_o - loss_t.item()) <= 1e-12 * abs(loss_t.item())
    assert _rel(g_o, g_t) <= 1e-10
    # the rounding is visible: the same objective without it is far from both
    _, g64, _ = _oracle_grad(pb)
    assert _rel(g64, g_t) > 1e-4


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_decided_gradient_matches_torch_with_fixed_pieces(seed):
    pb = _problem(seed, R=48, S=8)
    _, _, decisions = _torch_loss(pb, "bf16")      # decisions of torch's own BF16 forward
    loss_t, leaves, _ = _torch_loss(pb, "fixed", decisions)
    loss_t.backward()
    g_t = _flat(leaves)
    _, g_o, fw = _oracle_grad(pb, decide=oracle.bf16_round)
    assert _rel(g_o, g_t) <= 1e-10
    # the decided masks are the BF16 forward's, and some differ from the FP64 forward's
    for m_o, m_t in zip(fw["masks"], decisions[0]):
        assert np.array_equal(m_o, m_t.numpy())
    _, _, fw64 = _oracle_grad(pb)
    assert any(np.any(a != b) for a, b in zip(fw["masks"], fw64["masks"])), \
        "problem has no ReLU decision that BF16 and FP64 take differently"
