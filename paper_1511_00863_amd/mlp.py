"""The start-vector network on the device: parameters, training step, inference.

Thin marshalling over the ed_mlp_* entry points of include/ed.h; every
arithmetic step runs in the library's kernels (bfloat16 matrix cores with
float32 accumulation, float32 Adam).
"""

import ctypes
from ctypes import byref, c_double, c_float, c_int32, c_int64

import numpy as np
import torch

from ._ffi import ED_MLP_NPARAM, check, lib
from .api import _dptr, _stream

SHAPES = ((128, 32), (128,), (128, 128), (128,), (128, 128), (128,), (1, 128), (1,))


def flatten(ws, bs) -> np.ndarray:
    parts = []
    for w, b in zip(ws, bs):
        parts += [np.asarray(w, dtype=np.float64).ravel(), np.asarray(b, dtype=np.float64).ravel()]
    flat = np.concatenate(parts)
    assert flat.size == ED_MLP_NPARAM
    return flat


def unflatten(flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, k = [], 0
    for shp in SHAPES:
        n = int(np.prod(shp))
        out.append(flat[k:k + n].reshape(shp))
        k += n
    return out[0::2], out[1::2]


class StartVectorNet:
    """float32 master parameters, Adam moments and a minibatch workspace on the device."""

    def __init__(self, flat_params, device="cuda:0", batch: int = 4096):
        self.device = torch.device(device)
        self.params = torch.from_numpy(np.asarray(flat_params, dtype=np.float32)).to(self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.step_count = 0
        self.batch = int(batch)
        nb = c_int64(0)
        check(lib().ed_mlp_workspace_size(self.batch, byref(nb)))
        self.ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)

    @classmethod
    def from_init(cls, ws, bs, **kw):
        return cls(flatten(ws, bs), **kw)

    def numpy_params(self):
        return unflatten(self.params.double().cpu().numpy())

    def forward(self, st_up, st_dn, idx, out=None, stream=None):
        """psi for the states (st_up[idx[k,0]], st_dn[idx[k,1]]), k < n; keeps activations."""
        n = idx.shape[0]
        if n > self.batch:
            raise ValueError("minibatch larger than the workspace")
        idx = idx.to(torch.int32).contiguous()
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=self.device)
        check(lib().ed_mlp_forward(_dptr(self.params), _dptr(st_up), _dptr(st_dn), _dptr(idx), n, _dptr(out),
                                   _dptr(self.ws), _stream(stream)))
        return out

    def backward(self, target, stream=None):
        """Gradient of the mean squared error of the last forward into self.grad; loss on the device."""
        n = target.shape[0]
        check(lib().ed_mlp_backward(_dptr(self.params), _dptr(target.contiguous()), n, _dptr(self.grad),
                                    _dptr(self.loss), _dptr(self.ws), _stream(stream)))
        return self.grad

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step_count += 1
        check(lib().ed_mlp_adam(_dptr(self.params), _dptr(self.grad), _dptr(self.m), _dptr(self.v),
                                self.step_count, c_float(lr), c_float(beta1), c_float(beta2), c_float(eps),
                                _stream(stream)))

    def start_vector(self, ham, out=None, stream=None):
        """psi_theta over every state of ham, in ham's dtype (the proposed Lanczos start)."""
        if out is None:
            out = ham.empty_vec()
        h = ham.c_struct()
        check(lib().ed_mlp_start_vector(_dptr(self.params), byref(h), _dptr(out), _stream(stream)))
        return out


def row_cdf(psi, ham, stream=None):
    cdf = torch.empty(ham.dim_up + 1, dtype=torch.float64, device=psi.device)
    h = ham.c_struct()
    check(lib().ed_mlp_row_cdf(_dptr(psi), byref(h), _dptr(cdf), _stream(stream)))
    return cdf


def sample(psi, ham, cdf, uniforms, stream=None):
    """Minibatch (idx [n,2] int32, target [n] float32) drawn from the ground state psi."""
    n = uniforms.shape[0]
    idx = torch.empty((n, 2), dtype=torch.int32, device=psi.device)
    tgt = torch.empty(n, dtype=torch.float32, device=psi.device)
    h = ham.c_struct()
    check(lib().ed_mlp_sample(_dptr(psi), byref(h), _dptr(cdf), _dptr(uniforms.contiguous()), n, _dptr(idx),
                              _dptr(tgt), _stream(stream)))
    return idx, tgt


def neel_index(ham, lx: int = 4, ly: int = 4) -> int:
    """Vector index of the Neel state (up on sites with x+y even, down on the rest) when both
    fillings are half of the sites, else 0."""
    from .api import state_rank
    n_sites = lx * ly
    if ham.up.n_part != n_sites // 2 or ham.dn.n_part != n_sites - n_sites // 2:
        return 0
    up = sum(1 << (x + lx * y) for y in range(ly) for x in range(lx) if (x + y) % 2 == 0)
    dn = ((1 << n_sites) - 1) ^ up
    iu = int(state_rank(n_sites, ham.up.n_part, np.array([up], dtype=np.uint64))[0])
    idn = int(state_rank(n_sites, ham.dn.n_part, np.array([dn], dtype=np.uint64))[0])
    return iu * ham.dim_dn + idn


def train(net, data, uniforms, iters, lr=1e-3, lr_final=None, log_every=0):
    """Adam steps on minibatches cycling over the training ground states.

    data: list of (ham, psi, cdf) on the device; uniforms: device tensor
    [iters, batch, 2] of seeded uniforms.  lr_final: if given, the step size
    decays geometrically from lr to lr_final over the run.  Returns the loss
    after each step (host)."""
    losses = torch.empty(iters, dtype=torch.float64, device=net.device)
    for it in range(iters):
        ham, psi, cdf = data[it % len(data)]
        idx, tgt = sample(psi, ham, cdf, uniforms[it])
        net.forward(ham.up.dev_states, ham.dn.dev_states, idx)
        net.backward(tgt)
        step_lr = lr if lr_final is None else lr * (lr_final / lr) ** (it / max(1, iters - 1))
        net.adam(step_lr)
        losses[it:it + 1].copy_(net.loss)
    return losses.cpu().numpy()
