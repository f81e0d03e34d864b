"""Pins of the oracle's start-vector network: bf16 rounding, backward, Adam."""

import numpy as np
import pytest
import torch

from oracle import mlp
from synth import MLP_SIZES, mlp_init


def test_param_count():
    ws, bs = mlp_init(0)
    assert sum(w.size for w in ws) + sum(b.size for b in bs) == 37377


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8,
                                  0.0, -0.0, 65504.0, 1e-40])])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x32.astype(np.float64)), ref)


def test_features():
    f = mlp.features(np.array([0b101], dtype=np.uint64), np.array([1 << 15], dtype=np.uint64))
    assert f.shape == (1, 32)
    assert f[0, 0] == 1 and f[0, 1] == -1 and f[0, 2] == 1 and f[0, 16] == -1 and f[0, 31] == 1


def test_backward_finite_differences():
    rng = np.random.default_rng(1)
    sizes = (32, 16, 12, 8, 1)
    ws, bs = mlp_init(3, sizes)
    bs = [rng.normal(size=b.shape) * 0.1 for b in bs]
    x = 2.0 * rng.integers(0, 2, (9, 32)) - 1.0
    tgt = rng.normal(size=9)

    def L(ws_, bs_):
        out, _ = mlp.forward(ws_, bs_, x)
        return mlp.loss(out, tgt)

    out, cache = mlp.forward(ws, bs, x)
    gws, gbs = mlp.backward(ws, cache, out, tgt)
    h = 1e-6
    for l in range(len(ws)):
        for (i, j) in [(0, 0), (ws[l].shape[0] - 1, ws[l].shape[1] - 1), (ws[l].shape[0] // 2, 3)]:
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][i, j] += h
            wm[l][i, j] -= h
            fd = (L(wp, bs) - L(wm, bs)) / (2 * h)
            assert abs(fd - gws[l][i, j]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9
        bp = [b.copy() for b in bs]
        bm = [b.copy() for b in bs]
        bp[l][0] += h
        bm[l][0] -= h
        fd = (L(ws, bp) - L(ws, bm)) / (2 * h)
        assert abs(fd - gbs[l][0]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9


def test_backward_matches_autograd():
    rng = np.random.default_rng(2)
    ws, bs = mlp_init(4)
    x = 2.0 * rng.integers(0, 2, (64, 32)) - 1.0
    tgt = rng.normal(size=64)
    out, cache = mlp.forward(ws, bs, x)
    gws, gbs = mlp.backward(ws, cache, out, tgt)
    tw = [torch.tensor(w, requires_grad=True) for w in ws]
    tb = [torch.tensor(b, requires_grad=True) for b in bs]
    h = torch.tensor(x)
    for l in range(4):
        h = h @ tw[l].T + tb[l]
        if l < 3:
            h = torch.relu(h)
    ((h[:, 0] - torch.tensor(tgt)) ** 2).mean().backward()
    for l in range(4):
        assert np.allclose(gws[l], tw[l].grad.numpy(), rtol=1e-12, atol=1e-14)
        assert np.allclose(gbs[l], tb[l].grad.numpy(), rtol=1e-12, atol=1e-14)


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    p0 = [rng.normal(size=(4, 3)), rng.normal(size=5)]
    tp = [torch.tensor(p, requires_grad=True) for p in p0]
    opt = torch.optim.Adam(tp, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p = [x.copy() for x in p0]
    m = [np.zeros_like(x) for x in p0]
    v = [np.zeros_like(x) for x in p0]
    for step in range(1, 6):
        g = [rng.normal(size=x.shape) for x in p0]
        for t, gg in zip(tp, g):
            t.grad = torch.tensor(gg)
        opt.step()
        p, m, v = mlp.adam_step(p, g, m, v, step)
    for a, t in zip(p, tp):
        assert np.allclose(a, t.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_bf16_forward_close_to_exact():
    ws, bs = mlp_init(6)
    rng = np.random.default_rng(6)
    x = 2.0 * rng.integers(0, 2, (128, 32)) - 1.0
    a, _ = mlp.forward(ws, bs, x, bf16=False)
    b, _ = mlp.forward(ws, bs, x, bf16=True)
    assert np.linalg.norm(a - b) <= 3e-2 * np.linalg.norm(a)


def test_bf16_hand_computed_two_layer():
    """A 2-2-1 network whose every bf16 rounding is worked out by hand (bf16 keeps 8 significant bits,
    round to nearest, ties to even).  A rounding left out, or applied at a different place, moves the
    output or a gradient away from these exact binary fractions.

    Forward: z1 = r(x) r(W1)^T + b1, h1 = relu(z1), out = r(h1) r(W2)^T + b2.
      r(1 + 2^-8 + 2^-12) = 1 + 2^-7 (above the half-way point), r(0.75) = 0.75,
      r(0.5 + 2^-10) = 0.5 (a quarter spacing), r(-(1 + 3 2^-8)) = -(1 + 2^-6) (a tie: to the even 1 + 2^-6)
      z1 = [1 + 2^-7 - 0.75 + 7 2^-11, 0.5 + 1 + 2^-6 + 0.2] = [535 2^-11, 1.715625]
      r(535 2^-11 = 1000010111b 2^-11) = 536 2^-11 = 0.26171875 (above half), r(1.715625) = 220 2^-7 = 1.71875
      r(0.5 + 3 2^-10) = 0.5 + 2^-8, r(-(0.25 + 2^-12)) = -0.25
      out = 0.26171875 (0.5 + 2^-8) - 1.71875 / 4 + 0.1 = -0.1978057861328125 (+ the rounding of 0.1)
    Backward, target 0.15: g2 = 2 (out - 0.15) = -0.695611572265625, r(g2) = -178 2^-8 = -0.6953125
      dW2 = r(g2) r(h1) = [-0.181976318359375, -1.195068359375], db2 = g2
      g1 = r(g2) r(W2) = [-0.350372314453125, 0.173828125] (both z1 > 0)
      r(g1) = [-179 2^-9, 178 2^-10] = [-0.349609375, 0.173828125]
      dW1 = r(g1)^T r(x) = [[-0.349609375, 0.349609375], [0.173828125, -0.173828125]], db1 = g1
    """
    x = np.array([[1.0, -1.0]])
    ws = [np.array([[1 + 2 ** -8 + 2 ** -12, 0.75], [0.5 + 2 ** -10, -(1 + 3 * 2 ** -8)]]),
          np.array([[0.5 + 3 * 2 ** -10, -(0.25 + 2 ** -12)]])]
    bs = [np.array([7 * 2 ** -11, 0.2]), np.array([0.1])]
    out, cache = mlp.forward(ws, bs, x, bf16=True)
    assert abs(out[0] - (-0.1978057861328125)) <= 1e-15
    gws, gbs = mlp.backward(ws, cache, out, np.array([0.15]), bf16=True)
    assert np.allclose(gws[1], [[-0.181976318359375, -1.195068359375]], rtol=0, atol=1e-15)
    assert abs(gbs[1][0] - (-0.695611572265625)) <= 1e-15
    assert np.allclose(gws[0], [[-0.349609375, 0.349609375], [0.173828125, -0.173828125]], rtol=0, atol=1e-15)
    assert np.allclose(gbs[0], [-0.350372314453125, 0.173828125], rtol=0, atol=1e-15)
    # the same network without rounding gives other values (the pin can fail)
    out_x, _ = mlp.forward(ws, bs, x, bf16=False)
    assert abs(out_x[0] - out[0]) > 1e-4
