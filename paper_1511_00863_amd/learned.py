"""Learned Lanczos start vectors and time-to-E0 comparisons.

The method proposes its own training data: ground-state vectors from the
two-pass Lanczos run (ed_ground_state) at a set of training U values.  The
network is trained on minibatches drawn from them and then evaluated over all
states at a held-out U to give the start vector f_1 of Alg. 1.  If that
vector has zero or non-finite norm the seeded random start is used instead.
The reference energy of every run is that of converged plain float64 Lanczos.

Host code here only orchestrates calls into the library; all arithmetic runs
in its kernels (Lanczos, network, sampling) or in its host C++ (bisection).
"""

import time

import numpy as np
import torch

from . import api, mlp
from ._ffi import EdError
from synth import minibatch_uniforms, mlp_init, start_vector


def _random_start(ham, seed):
    return torch.from_numpy(start_vector(seed, ham.dim)).to(ham.device, ham.torch_dtype)


def reference_energy(up, dn, t, U, seed, tol=1e-12, max_steps=800, tile=None):
    """Converged plain float64 Lanczos from the seeded random start."""
    h = api.Hamiltonian(up, dn, t, U, "f64")
    api.apply_tuned_tile(h, tune_if_missing=False)
    r = h.ground_energy(_random_start(h, seed), max_steps, tol=tol, check_every=15)
    return r["e0"], r["steps"]


def training_data(up, dn, t, us, seed=100, dtype="f32", tol=1e-9, extra_steps=20, max_steps=800, gauge=None):
    """(ham, psi, cdf) per training U: the two-pass vector, pass 1 run until E0 settles to tol plus
    extra_steps more (at most max_steps)."""
    out = []
    for k, U in enumerate(us):
        h = api.Hamiltonian(up, dn, t, U, dtype)
        api.apply_tuned_tile(h, tune_if_missing=False)
        x = _random_start(h, seed + k)
        gi = mlp.neel_index(h) if gauge is None else gauge
        # pass 1 runs until E0 settles to tol, then extra_steps more (at most max_steps); pass 2 builds psi
        e0, steps, psi = h.ground_state(x, max_steps, gauge_index=gi, tol=tol, extra=extra_steps)
        del x
        out.append((h, psi, mlp.row_cdf(psi, h)))
    return out


def train_network(data, iters=1500, batch=4096, seed=7, init_seed=3, lr=1e-3, lr_final=None):
    ws, bs = mlp_init(init_seed)
    net = mlp.StartVectorNet.from_init(ws, bs, batch=batch, device=data[0][1].device)
    uni = torch.from_numpy(minibatch_uniforms(seed, iters, batch)).to(data[0][1].device)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = mlp.train(net, data, uni, iters, lr=lr, lr_final=lr_final)
    torch.cuda.synchronize()
    return net, losses, time.perf_counter() - t0


def steps_to_accuracy(a, b, e_ref, rel_tol):
    """First j with |E0(j) - E_ref| <= rel_tol |E_ref| (host bisection of T_j), or None."""
    for j in range(1, len(a) + 1):
        e = api.tridiag_lowest(a[:j], b[1:j])
        if abs(e - e_ref) <= rel_tol * abs(e_ref):
            return j
    return None


def time_to_e0(ham, f1_fn, e_ref, rel_tol, max_steps=600, reps=1):
    """Steps and wall time to reach E0 within rel_tol of the reference from the start f1_fn().

    The run length is found once from the coefficients; the timed region then
    covers producing f1 (network inference for a learned start; a copy of a
    resident vector for a random start) plus exactly that many steps."""
    f1 = f1_fn()
    probe = ham.ground_energy(f1, max_steps, tol=0.0, check_every=30)
    k = steps_to_accuracy(probe["a"], probe["b"], e_ref, rel_tol)
    if k is None:
        return {"steps": None, "ms": None}
    del f1
    best = None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f1 = f1_fn()
        r = ham.ground_energy(f1, k, tol=0.0, check_every=k)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) * 1e3
        best = dt if best is None else min(best, dt)
        del f1
    return {"steps": k, "ms": best, "e0": r["e0"]}


def learned_start(net, ham, seed):
    """The network's vector over all states, or the seeded random start if it is unusable."""
    f1 = net.start_vector(ham)
    run = api.LanczosRun(ham, 1)
    try:
        run.init(f1)          # rejects zero or non-finite norms
        return f1, "network"
    except EdError:
        return _random_start(ham, seed), "random-fallback"
