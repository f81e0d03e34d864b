"""The batched persistent launch: every instance agrees with its own solo run."""

import numpy as np
import pytest
import torch

import paper_1511_00863_amd as ed
from synth import batch_instances, ring_bonds, start_vector, torus_bonds
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _solo_e0(up, dn, U, seed, dtype, tol):
    h = ed.Hamiltonian(up, dn, 1.0, U, dtype)
    x = torch.from_numpy(start_vector(seed, h.dim)).to("cuda:0", h.torch_dtype)
    r = h.ground_energy(x, 600, tol=tol, check_every=12)
    return r["e0"], r["steps"]


def test_batch_mixed_shapes():
    bonds = torus_bonds(4, 4)
    tabs = {n: ed.SpinTables(16, bonds, n, "cuda:0") for n in (2, 3, 4)}
    ring = ed.SpinTables(8, ring_bonds(8), 4, "cuda:0")
    spec = [(tabs[3], tabs[3], 0.0, 11), (tabs[3], tabs[3], 4.0, 12), (tabs[2], tabs[4], 2.0, 13),
            (tabs[4], tabs[2], 8.0, 14), (ring, ring, 4.0, 15), (tabs[2], tabs[2], 1.0, 16)]
    hams = [ed.Hamiltonian(u, d, 1.0, U, "f32") for (u, d, U, s) in spec]
    f1s = [torch.from_numpy(start_vector(s, h.dim)).to("cuda:0", torch.float32) for h, (_, _, _, s) in zip(hams, spec)]
    announce("batch mixed shapes n=%d" % len(hams))
    r = ed.ground_energy_batch(hams, f1s, 400, tol=1e-7)
    # at U = 0 the many-body spectrum has few distinct levels, so the Krylov space
    # closes early: a breakdown there is the exact answer, not a failure
    assert np.isin(r["status"], (ed.ED_OK, ed.ED_BREAKDOWN)).all(), r["status"]
    assert (r["status"][1:] == ed.ED_OK).all(), r["status"]
    for k, (u, d, U, s) in enumerate(spec):
        e64, _ = _solo_e0(u, d, U, s, "f64", 1e-12)
        assert abs(r["e0"][k] - e64) <= 1e-6 * abs(e64), (k, r["e0"][k], e64)
        assert abs(r["e0_device"][k] - r["e0"][k]) <= 1e-9 * abs(e64)
    # U = 0, 3+3 on the 4x4 torus: band sum -16
    assert abs(r["e0"][0] - (-16.0)) <= 1e-6 * 16


@pytest.mark.parametrize("solo_dim", [0, ed.api.BATCH_SOLO_DIM], ids=["persistent", "scheduled"])
def test_batch_64_uneven_fillings(solo_dim):
    """64 instances, U ~ U[0,8], N_up = N_dn in {3,4,5,6}, |dE0| < 1e-6: all in one persistent launch
    (solo_dim 0), or with the instances of at least 2^22 states (5 and 6 per species) run one by one after
    it."""
    bonds = torus_bonds(4, 4)
    draws = batch_instances(64, 1000)
    tabs = {n: ed.SpinTables(16, bonds, n, "cuda:0") for n in (3, 4, 5, 6)}
    hams = [ed.Hamiltonian(tabs[n], tabs[n], 1.0, U, "f32") for (U, n, s) in draws]
    for h in hams:
        ed.api.apply_tuned_tile(h, tune_if_missing=False)
    f1s = [torch.from_numpy(start_vector(s, h.dim)).to("cuda:0", torch.float32) for h, (U, n, s) in zip(hams, draws)]
    announce("batch 64 uneven, total dim %d, solo_dim %d" % (sum(h.dim for h in hams), solo_dim))
    r = ed.ground_energy_batch(hams, f1s, 500, tol=1e-6, solo_dim=solo_dim)
    assert (r["status"] == ed.ED_OK).all(), r["status"]
    solo = np.array([solo_dim > 0 and h.dim >= solo_dim for h in hams])
    assert solo.sum() == (0 if solo_dim == 0 else sum(n >= 5 for (U, n, s) in draws))
    assert np.array_equal(r["e0_device"][solo], r["e0"][solo])   # one-by-one items report the host value
    assert (r["steps"] > 0).all()
    del f1s
    torch.cuda.empty_cache()
    # every instance against its solo float64 energy (sample 8 to bound the run time)
    for k in [0, 5, 17, 23, 31, 42, 50, 63]:
        U, n, s = draws[k]
        e64, _ = _solo_e0(tabs[n], tabs[n], U, s, "f64", 1e-11)
        assert abs(r["e0"][k] - e64) <= 1e-6 * abs(e64), (k, U, n, r["e0"][k], e64)


def test_batch_every_item_one_by_one():
    """solo_dim = 1 sends every item through the one-instance run (no persistent launch): the same E0 as the
    persistent launch to 1e-6, coefficients written to each item's a and b, no phase times."""
    bonds = torus_bonds(4, 4)
    draws = batch_instances(6, 4000, fillings=(2, 3))
    tabs = {n: ed.SpinTables(16, bonds, n, "cuda:0") for n in (2, 3)}
    hams = [ed.Hamiltonian(tabs[n], tabs[n], 1.0, U, "f32") for (U, n, s) in draws]
    f1s = [torch.from_numpy(start_vector(s, h.dim)).to("cuda:0", torch.float32) for h, (U, n, s) in zip(hams, draws)]
    announce("batch, every item one by one")
    ra = ed.ground_energy_batch(hams, f1s, 400, tol=1e-7, solo_dim=1)
    rb = ed.ground_energy_batch(hams, f1s, 400, tol=1e-7, solo_dim=0)
    assert (ra["status"] == ed.ED_OK).all() and (rb["status"] == ed.ED_OK).all(), (ra["status"], rb["status"])
    assert not ra["graph_used"] and all(v == 0.0 for v in ra["phase_ms"].values())
    assert np.max(np.abs(ra["e0"] - rb["e0"]) / np.abs(rb["e0"])) <= 1e-6
    assert np.array_equal(ra["e0_device"], ra["e0"])
