"""Parity of the device occupation moments (diagonal observables of a state) with the oracle."""

import numpy as np
import pytest
import torch

import paper_1511_00863_amd as ed
from oracle.observables import correlations, occupation_moments
from oracle.hamiltonian import Model
from paper_1511_00863_amd import mlp
from synth import complete_bonds, ring_bonds, torus_bonds
from tests.gpu_util import announce, ham, seeded_start

pytestmark = pytest.mark.gpu

CASES = [
    ("ring8_3x2", 8, ring_bonds(8), 3, 2),
    ("t44_3x3", 16, torus_bonds(4, 4), 3, 3),
    ("ring6_0x3", 6, ring_bonds(6), 0, 3),
    ("complete12_5x6", 12, complete_bonds(12), 5, 6),
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_moments_match_oracle(case, dtype):
    name, ns, bonds, nu, nd = case
    h = ham(ns, bonds, nu, nd, 1.0, 2.0, dtype)
    x_host, x = seeded_start(51, h.dim, dtype)       # the oracle sees the same (rounded) values
    announce("occupation moments %s %s" % (name, dtype))
    g = h.occupation_moments(x, ns)
    # the device normalises by sum_x |psi_x|^2; the oracle's definition is the raw weighted sum
    ref = occupation_moments(x_host, h.up.states, h.dn.states, ns) / np.sum(x_host ** 2)
    assert np.max(np.abs(g - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
    got, want = ed.occupation_correlations(g, ns), correlations(ref, ns)
    for k in ("docc", "nn", "szsz"):
        assert np.max(np.abs(got[k] - want[k])) <= 1e-12


def test_zero_vector_and_bad_sites_rejected():
    h = ham(8, ring_bonds(8), 3, 2, 1.0, 2.0, "f64")
    z = torch.zeros(h.dim, dtype=torch.float64, device="cuda:0")
    announce("occupation moments of a zero vector")
    assert np.all(h.occupation_moments(z, 8) == 0.0)
    with pytest.raises(ed.EdError):
        h.occupation_moments(z, 33)


def test_hellmann_feynman_t44_4x4():
    """dE0/dU = sum_i <n_i,up n_i,dn>: double occupancy of the device ground state against a finite
    difference of device ground-state energies (4x4 torus, 4+4, U = 4)."""
    tab = ed.SpinTables(16, torus_bonds(4, 4), 4, "cuda:0")
    U, dU = 4.0, 1e-3
    e = {}
    for u in (U - dU, U + dU):
        hh = ed.Hamiltonian(tab, tab, 1.0, u, "f64")
        _, x = seeded_start(52, hh.dim, "f64")
        announce("ground energy 4x4 4+4 U=%g" % u)
        e[u] = hh.ground_energy(x, 400, tol=1e-13, check_every=10)["e0"]
    h = ed.Hamiltonian(tab, tab, 1.0, U, "f64")
    _, x = seeded_start(52, h.dim, "f64")
    r = h.ground_energy(x, 400, tol=1e-13, check_every=10)
    announce("ground state 4x4 4+4 U=4")
    e0, steps, psi = h.ground_state(x, r["steps"] + 20, gauge_index=mlp.neel_index(h))
    c = ed.occupation_correlations(h.occupation_moments(psi, 16), 16)
    fd = (e[U + dU] - e[U - dU]) / (2 * dU)
    assert abs(c["docc"].sum() - fd) <= 1e-5 * abs(fd)
    # translation invariance of the torus; densities N/N_s per species
    assert np.ptp(c["docc"]) <= 1e-8


def test_full_size_sum_rules_t44_8x8():
    """At the benchmark size (4x4, 8+8, D = 165,636,900): sum rules that hold for any state, and the
    symmetries of the ground state (half filling on a translation-invariant lattice)."""
    tab = ed.SpinTables(16, torus_bonds(4, 4), 8, "cuda:0")
    h = ed.Hamiltonian(tab, tab, 1.0, 4.0, "f32")
    ed.api.apply_tuned_tile(h, tune_if_missing=False)
    _, x = seeded_start(5, h.dim, "f32")
    announce("ground state 4x4 8+8 mixed")
    r = h.ground_energy(x, 300, tol=1e-7, check_every=15)
    e0, steps, psi = h.ground_state(x, r["steps"] + 20, gauge_index=mlp.neel_index(h))
    del x
    announce("occupation moments 4x4 8+8")
    g = h.occupation_moments(psi, 16)
    c = ed.occupation_correlations(g, 16)
    n_up, n_dn = np.diag(g)[:16], np.diag(g)[16:]
    assert abs(n_up.sum() - 8) < 1e-9 and abs(n_dn.sum() - 8) < 1e-9
    n_i = n_up + n_dn
    assert np.max(np.abs(c["nn"].sum(axis=1) - 16 * n_i)) < 1e-8          # sum_j n_j = N
    assert np.max(np.abs(c["szsz"].sum(axis=1))) < 1e-8                    # S^z_tot = 0
    assert np.max(np.abs(n_up - 0.5)) < 1e-4 and np.ptp(c["docc"]) < 1e-4  # uniform at half filling
    assert 0.0 < c["docc"][0] < 0.25                                      # U > 0 suppresses double occupancy


FLIP_CASES = [
    ("ring8_3x2", 8, ring_bonds(8), 3, 2),
    ("ring8_4x4", 8, ring_bonds(8), 4, 4),
    ("t32_3x2", 6, torus_bonds(3, 2), 3, 2),
    ("ring6_0x3", 6, ring_bonds(6), 0, 3),
    ("ring18_2x2", 18, ring_bonds(18), 2, 2),     # more than 16 sites: the 32-site kernel variant
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", FLIP_CASES, ids=[c[0] for c in FLIP_CASES])
def test_spin_flip_moments_match_oracle(case, dtype):
    from oracle.observables import spin_flip_moments
    name, ns, bonds, nu, nd = case
    h = ham(ns, bonds, nu, nd, 1.0, 2.0, dtype)
    x_host, x = seeded_start(53, h.dim, dtype)
    announce("spin-flip moments %s %s" % (name, dtype))
    c = h.spin_flip_moments(x, ns)
    ref = spin_flip_moments(x_host, h.up.states, h.dn.states, ns) / np.sum(x_host ** 2)
    assert np.max(np.abs(c - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_full_size_singlet_t44_8x8():
    """4x4 torus at half filling (D = 165,636,900): the float64 ground state is a singlet, so the spin-flip
    moments (one kernel) equal twice the S^z correlations (another) off the diagonal, and sum <S_i . S_j> = 0."""
    tab = ed.SpinTables(16, torus_bonds(4, 4), 8, "cuda:0")
    h = ed.Hamiltonian(tab, tab, 1.0, 4.0, "f64")
    ed.api.apply_tuned_tile(h, tune_if_missing=False)
    _, x = seeded_start(5, h.dim, "f64")
    announce("ground state 4x4 8+8 f64")
    r = h.ground_energy(x, 400, tol=1e-12, check_every=15)
    e0, steps, psi = h.ground_state(x, r["steps"] + 30, gauge_index=mlp.neel_index(h))
    del x
    announce("spin correlations 4x4 8+8")
    g = h.occupation_moments(psi, 16)
    c = h.spin_flip_moments(psi, 16)
    zz = ed.occupation_correlations(g, 16)["szsz"]
    off = ~np.eye(16, dtype=bool)
    assert np.max(np.abs(c[off] - 2.0 * zz[off])) < 1e-6
    ss = ed.spin_correlations(g, c, 16)
    assert abs(ss.sum()) < 1e-5
    assert np.all(ss[0, [1, 4]] < 0.0)      # antiferromagnetic nearest neighbours


BOND_CASES = [
    ("ring8_3x2", 8, ring_bonds(8), 3, 2),
    ("t32_3x3", 6, torus_bonds(3, 2), 3, 3),
    ("ring6_0x3", 6, ring_bonds(6), 0, 3),
    ("complete8_3x3", 8, complete_bonds(8), 3, 3),     # 28 bonds: two groups of 16
]


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("case", BOND_CASES, ids=[c[0] for c in BOND_CASES])
def test_bond_moments_match_oracle(case, dtype):
    from oracle.observables import bond_moments
    name, ns, bonds, nu, nd = case
    h = ham(ns, bonds, nu, nd, 1.0, 2.0, dtype)
    x_host, x = seeded_start(54, h.dim, dtype)
    announce("bond moments %s %s" % (name, dtype))
    k = h.bond_moments(x, ns, bonds)
    ref = bond_moments(x_host, h.up.states, h.dn.states, ns, bonds) / np.sum(x_host ** 2)
    assert np.max(np.abs(k - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_full_size_energy_identity_t44_8x8():
    """4x4 8+8, float64 ground state: E0 = -t sum_b K_b + U sum_i <n_i,up n_i,dn> (bond kernel and occupation
    moments against the Lanczos energy), and the translation-invariant bonds carry equal energy."""
    bonds = torus_bonds(4, 4)
    tab = ed.SpinTables(16, bonds, 8, "cuda:0")
    h = ed.Hamiltonian(tab, tab, 1.0, 4.0, "f64")
    ed.api.apply_tuned_tile(h, tune_if_missing=False)
    _, x = seeded_start(5, h.dim, "f64")
    announce("ground state 4x4 8+8 f64 (bonds)")
    r = h.ground_energy(x, 400, tol=1e-12, check_every=15)
    e0, steps, psi = h.ground_state(x, r["steps"] + 30, gauge_index=mlp.neel_index(h))
    del x
    announce("bond moments 4x4 8+8")
    k = h.bond_moments(psi, 16, bonds)
    g = h.occupation_moments(psi, 16)
    energy = -1.0 * k.sum() + 4.0 * np.trace(g[:16, 16:])
    assert abs(energy - e0) <= 1e-8 * abs(e0), (energy, e0)
    assert np.ptp(k) < 1e-6 and np.max(np.abs(k[:, 0] - k[:, 1])) < 1e-8
