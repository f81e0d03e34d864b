"""What the trained start-vector network gains: fewer Lanczos steps to the reference E0 at held-out U."""

import numpy as np
import pytest
import torch

import paper_1511_00863_amd as ed
from paper_1511_00863_amd import learned
from synth import start_vector, torus_bonds
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def test_learned_start_beats_random_at_held_out_u():
    """4x4 torus, 4+4: train on ground states at U = 1..8, evaluate at U = 1.5, 3.5, 5.5, 7.5.
    Reference: converged plain float64 Lanczos.  Both starts run the mixed form to 1e-6."""
    tab = ed.SpinTables(16, torus_bonds(4, 4), 4, "cuda:0")
    announce("learned start: training data")
    data = learned.training_data(tab, tab, 1.0, [1, 2, 3, 4, 5, 6, 7, 8])
    announce("learned start: training")
    net, losses, _ = learned.train_network(data, iters=800, batch=2048)
    assert np.all(np.isfinite(losses))
    gains = []
    for U in (1.5, 3.5, 5.5, 7.5):
        announce("learned start: held-out U=%g" % U)
        e_ref, _ = learned.reference_energy(tab, tab, 1.0, U, 5)
        h = ed.Hamiltonian(tab, tab, 1.0, U, "f32")
        x = torch.from_numpy(start_vector(5, h.dim)).to("cuda:0", torch.float32)
        rnd = learned.time_to_e0(h, lambda: x.clone(), e_ref, 1e-6)
        lrn = learned.time_to_e0(h, lambda: learned.learned_start(net, h, 5)[0], e_ref, 1e-6)
        assert rnd["steps"] is not None and lrn["steps"] is not None
        assert abs(lrn["e0"] - e_ref) <= 1e-6 * abs(e_ref)
        gains.append(rnd["steps"] - lrn["steps"])
    assert min(gains) > 0, gains


def test_fallback_to_random_start():
    """An all-zero network proposes the zero vector; the seeded random start is used instead."""
    from paper_1511_00863_amd import mlp
    tab = ed.SpinTables(16, torus_bonds(4, 4), 3, "cuda:0")
    h = ed.Hamiltonian(tab, tab, 1.0, 2.0, "f32")
    net = mlp.StartVectorNet(np.zeros(ed._ffi.ED_MLP_NPARAM), batch=64)
    announce("learned start fallback")
    f1, kind = learned.learned_start(net, h, 5)
    assert kind == "random-fallback"
    r = h.ground_energy(f1, 200, tol=1e-7)
    assert r["status"] == ed.ED_OK


def test_learned_start_at_half_filling_8x8():
    """The configured size: 4x4 torus at 8 + 8 (dim 165,636,900).  The network trains on two-pass
    ground states at U = 1..8 (3000 Adam steps of 4096 samples, as the benchmark) and proposes f_1 at the
    held-out U = 3.5; the mixed form from it reaches the converged float64 reference E0 to 1e-6 in fewer
    steps than from the seeded random start."""
    up = ed.SpinTables(16, torus_bonds(4, 4), 8, "cuda:0")
    announce("learned start 8+8: training data (8 ground states)")
    data = learned.training_data(up, up, 1.0, [1, 2, 3, 4, 5, 6, 7, 8])
    announce("learned start 8+8: training")
    net, losses, _ = learned.train_network(data, iters=3000, batch=4096)
    del data
    torch.cuda.empty_cache()
    assert np.all(np.isfinite(losses)) and losses[-20:].mean() < losses[:20].mean()
    U = 3.5
    announce("learned start 8+8: held-out U=%g" % U)
    e_ref, _ = learned.reference_energy(up, up, 1.0, U, 5)
    h = ed.Hamiltonian(up, up, 1.0, U, "f32")
    ed.api.apply_tuned_tile(h, tune_if_missing=False)
    x = torch.from_numpy(start_vector(5, h.dim)).to("cuda:0", torch.float32)
    rnd = learned.time_to_e0(h, lambda: x.clone(), e_ref, 1e-6)
    f1, kind = learned.learned_start(net, h, 5)
    assert kind == "network"
    del f1
    lrn = learned.time_to_e0(h, lambda: learned.learned_start(net, h, 5)[0], e_ref, 1e-6)
    assert rnd["steps"] is not None and lrn["steps"] is not None
    assert abs(lrn["e0"] - e_ref) <= 1e-6 * abs(e_ref)
    assert lrn["steps"] < rnd["steps"], (lrn["steps"], rnd["steps"])
