"""The start-vector network: float64 forward, backward and Adam.

Network psi(bits) with 32 inputs (16 up occupation bits, then 16 down bits,
each mapped to 2*bit - 1), three hidden layers of 128 with ReLU and one linear
output.  Loss: mean squared error against target amplitudes.  Adam with bias
correction.  With ``bf16=True`` every matmul operand (weights, layer inputs and
back-propagated gradients) is first rounded to bfloat16 (round to nearest even
on the top 16 bits of the float32 value), mirroring a device that multiplies
in bfloat16 and accumulates in float32; biases and accumulation stay float64.
"""

import numpy as np


def bf16_round(x) -> np.ndarray:
    """float64 -> float32 (nearest even) -> bfloat16 (nearest even) -> float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out = np.where(nan, np.nan, out)
    return out


def features(st_up, st_dn, n_bits: int = 16) -> np.ndarray:
    """(N, 32) inputs: 2*bit - 1 for up bits 0..15 then down bits 0..15."""
    su = np.asarray(st_up, dtype=np.uint64)
    sd = np.asarray(st_dn, dtype=np.uint64)
    cols = [((su >> np.uint64(k)) & np.uint64(1)).astype(np.float64) for k in range(n_bits)]
    cols += [((sd >> np.uint64(k)) & np.uint64(1)).astype(np.float64) for k in range(n_bits)]
    return 2.0 * np.stack(cols, axis=1) - 1.0


def _r(x, bf16):
    return bf16_round(x) if bf16 else np.asarray(x, dtype=np.float64)


def forward(ws, bs, x, bf16=False):
    """Returns (out (N,), cache).  ws[l] has shape (fan_out, fan_in)."""
    h = np.asarray(x, dtype=np.float64)
    acts, pre = [h], []
    n_layers = len(ws)
    for l in range(n_layers):
        z = _r(h, bf16) @ _r(ws[l], bf16).T + bs[l]
        pre.append(z)
        h = np.maximum(z, 0.0) if l < n_layers - 1 else z
        acts.append(h)
    return h[:, 0], {"acts": acts, "pre": pre}


def loss(out, target) -> float:
    d = np.asarray(out) - np.asarray(target)
    return float(np.mean(d * d))


def backward(ws, cache, out, target, bf16=False):
    """Gradients of the mean squared error w.r.t. every weight and bias."""
    acts, pre = cache["acts"], cache["pre"]
    n = out.shape[0]
    g = (2.0 / n) * (np.asarray(out) - np.asarray(target))[:, None]   # dL/dz of the last layer
    gws, gbs = [None] * len(ws), [None] * len(ws)
    for l in reversed(range(len(ws))):
        gr = _r(g, bf16)
        gws[l] = gr.T @ _r(acts[l], bf16)
        gbs[l] = g.sum(axis=0)
        if l > 0:
            dh = gr @ _r(ws[l], bf16)
            g = dh * (pre[l - 1] > 0.0)
    return gws, gbs


def adam_step(params, grads, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected) on lists of arrays; returns new (params, m, v)."""
    new_p, new_m, new_v = [], [], []
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = beta1 * mm + (1.0 - beta1) * g
        vv = beta2 * vv + (1.0 - beta2) * g * g
        mh = mm / (1.0 - beta1 ** step)
        vh = vv / (1.0 - beta2 ** step)
        new_p.append(p - lr * mh / (np.sqrt(vh) + eps))
        new_m.append(mm)
        new_v.append(vv)
    return new_p, new_m, new_v
