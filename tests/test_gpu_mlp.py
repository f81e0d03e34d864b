"""Parity of the bf16-MFMA start-vector network with the float64 oracle (bf16 operand rounding)."""

import numpy as np
import pytest
import torch

import paper_1511_00863_amd as ed
from paper_1511_00863_amd import mlp as dmlp
from oracle import mlp as omlp
from synth import mlp_init, ring_bonds, start_vector, torus_bonds
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-30))


@pytest.fixture(scope="module")
def setup():
    rng = np.random.default_rng(0)
    ws, bs = mlp_init(11)
    bs = [rng.normal(size=b.shape) * 0.1 for b in bs]          # nonzero biases so every term is exercised
    up = ed.SpinTables(16, torus_bonds(4, 4), 5, "cuda:0")
    dn = ed.SpinTables(16, torus_bonds(4, 4), 3, "cuda:0")
    n = 1000                                                   # not a multiple of 16 or 32: ragged tail
    iu = rng.integers(0, up.dim, n)
    idn = rng.integers(0, dn.dim, n)
    x = omlp.features(up.states[iu], dn.states[idn])
    tgt = rng.normal(size=n)
    net = dmlp.StartVectorNet.from_init(ws, bs, batch=1024)
    idx = torch.from_numpy(np.stack([iu, idn], 1).astype(np.int32)).cuda()
    return dict(ws=ws, bs=bs, up=up, dn=dn, x=x, tgt=tgt, net=net, idx=idx, n=n)


def test_forward_parity(setup):
    S = setup
    announce("mlp forward n=%d" % S["n"])
    out = S["net"].forward(S["up"].dev_states, S["dn"].dev_states, S["idx"]).double().cpu().numpy()
    ref, _ = omlp.forward(S["ws"], S["bs"], S["x"], bf16=True)
    # measured 1.1e-4: float32 against float64 accumulation, and the bf16 rounding of an activation
    # flipping where the two fall on either side of a rounding point
    assert _rel(out, ref) <= 3.5e-4
    exact, _ = omlp.forward(S["ws"], S["bs"], S["x"], bf16=False)
    assert _rel(out, exact) <= 1e-2     # measured 2.5e-3: bf16 operands against exact ones


def test_backward_parity(setup):
    S = setup
    net = S["net"]
    announce("mlp backward")
    out = net.forward(S["up"].dev_states, S["dn"].dev_states, S["idx"])
    tgt = torch.from_numpy(S["tgt"].astype(np.float32)).cuda()
    net.backward(tgt)
    gw, gb = dmlp.unflatten(net.grad.double().cpu().numpy())
    ref_out, cache = omlp.forward(S["ws"], S["bs"], S["x"], bf16=True)
    rw, rb = omlp.backward(S["ws"], cache, ref_out, S["tgt"].astype(np.float32).astype(np.float64), bf16=True)
    for l in range(4):   # measured at most 6.4e-5 (weights) and 3.2e-5 (biases)
        assert _rel(gw[l], rw[l]) <= 2e-4, ("W", l, _rel(gw[l], rw[l]))
        assert _rel(gb[l], rb[l]) <= 1e-4, ("b", l, _rel(gb[l], rb[l]))
    loss = float(net.loss.cpu()[0])
    assert abs(loss - omlp.loss(ref_out, S["tgt"])) <= 5e-5 * omlp.loss(ref_out, S["tgt"])   # measured 1.6e-5


def test_adam_parity(setup):
    S = setup
    rng = np.random.default_rng(3)
    flat = dmlp.flatten(S["ws"], S["bs"])
    net = dmlp.StartVectorNet(flat, batch=64)
    p = [flat.copy()]
    m = [np.zeros_like(flat)]
    v = [np.zeros_like(flat)]
    announce("mlp adam")
    for step in range(1, 4):
        g = rng.normal(size=flat.size).astype(np.float32)
        net.grad.copy_(torch.from_numpy(g))
        net.adam(lr=1e-3)
        p, m, v = omlp.adam_step(p, [g.astype(np.float64)], m, v, step)
    got = net.params.double().cpu().numpy()
    assert np.max(np.abs(got - p[0])) <= 1e-6 * max(1.0, np.max(np.abs(p[0])))


def test_start_vector_over_all_states(setup):
    S = setup
    h = ed.Hamiltonian(S["up"], S["dn"], 1.0, 2.0, "f32")
    announce("mlp start vector dim=%d" % h.dim)
    psi = S["net"].start_vector(h).double().cpu().numpy()
    rng = np.random.default_rng(5)
    ks = rng.integers(0, h.dim, 700)
    x = omlp.features(S["up"].states[ks // h.dim_dn], S["dn"].states[ks % h.dim_dn])
    ref, _ = omlp.forward(S["ws"], S["bs"], x, bf16=True)
    assert _rel(psi[ks], ref) <= 7.5e-5     # measured 2.5e-5
    h64 = ed.Hamiltonian(S["up"], S["dn"], 1.0, 2.0, "f64")
    psi64 = S["net"].start_vector(h64).cpu().numpy()
    assert np.array_equal(psi64.astype(np.float32), psi.astype(np.float32))


def test_sampling():
    tab = ed.SpinTables(6, ring_bonds(6), 3, "cuda:0")
    h = ed.Hamiltonian(tab, tab, 1.0, 4.0, "f64")
    rng = np.random.default_rng(1)
    psi_h = rng.normal(size=h.dim) * np.exp(-np.arange(h.dim) / 100.0)
    psi_h /= np.linalg.norm(psi_h)
    psi = torch.from_numpy(psi_h).cuda()
    announce("mlp sampling")
    cdf = dmlp.row_cdf(psi, h)
    rows = (psi_h.reshape(h.dim_up, h.dim_dn) ** 2).sum(1)
    assert np.allclose(cdf.cpu().numpy()[:-1], np.cumsum(rows) / rows.sum(), rtol=1e-12, atol=1e-14)
    n = 200000
    u = rng.random((n, 2))
    u[:, 0] = 0.25                     # all from |psi|^2
    idx, tgt = dmlp.sample(psi, h, cdf, torch.from_numpy(u).cuda())
    idx = idx.cpu().numpy()
    k = idx[:, 0] * h.dim_dn + idx[:, 1]
    assert np.allclose(tgt.cpu().numpy(), np.sqrt(h.dim) * psi_h[k], rtol=1e-6, atol=1e-7)
    freq = np.bincount(k, minlength=h.dim) / n
    p = psi_h ** 2
    big = p > 5e-3
    assert np.max(np.abs(freq[big] - p[big]) / np.sqrt(p[big] / n)) < 6.0   # within 6 sigma
    u[:, 0] = 0.75                     # uniform proposal
    idx, _ = dmlp.sample(psi, h, cdf, torch.from_numpy(u).cuda())
    k = idx.cpu().numpy()
    k = k[:, 0] * h.dim_dn + k[:, 1]
    assert np.array_equal(k, np.minimum((u[:, 1] * h.dim).astype(np.int64), h.dim - 1))


def test_training_reduces_loss():
    tab = ed.SpinTables(16, torus_bonds(4, 4), 3, "cuda:0")
    h = ed.Hamiltonian(tab, tab, 1.0, 4.0, "f32")
    x = torch.from_numpy(start_vector(7, h.dim)).to("cuda:0", torch.float32)
    announce("mlp training smoke")
    e0, steps, psi = h.ground_state(x, 120, gauge_index=0)
    cdf = dmlp.row_cdf(psi, h)
    ws, bs = mlp_init(3)
    net = dmlp.StartVectorNet.from_init(ws, bs, batch=512)
    from synth import minibatch_uniforms
    uni = torch.from_numpy(minibatch_uniforms(9, 300, 512)).cuda()
    losses = dmlp.train(net, [(h, psi, cdf)], uni, 300, lr=1e-3)
    assert np.all(np.isfinite(losses))
    assert losses[-20:].mean() < 0.7 * losses[:20].mean()
